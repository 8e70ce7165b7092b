/*
 * fluxlbm.h -- C ABI of the MI355X (gfx950) D3Q19 lattice-Boltzmann library
 * with the adaptive volumetric-flux inlet of McClure, Li, Sheppard and
 * Miller, "An Adaptive Volumetric Flux Boundary Condition for Lattice
 * Boltzmann Methods" (arXiv:1806.10589).
 *
 * What one time step computes (flbm_step):
 *   - pull streaming of the D3Q19 populations over a sparse list of pore
 *     sites (Methods, eq. LBE), with halfway bounce-back at solid voxels and
 *     at non-periodic side faces;
 *   - at the inlet plane z = 0: the uniform inlet density that makes the
 *     total volumetric flux equal the target, found by integrating the
 *     consistency condition over the inlet pore sites (Methods, eq. inlet,
 *     eq. flux, eq. potential), then the pressure condition with that
 *     density, closed with Hecht and Harting's transverse corrections
 *     (Appendix B);
 *   - at the outlet plane z = nz-1: the same pressure condition with a fixed
 *     density (Methods, last paragraph);
 *   - collision at every pore site: BGK (single fluid) or the colour-gradient
 *     two-fluid model of Appendix A;
 *   - per-step FP64 records of rho_in, Q_in, Q_out; total mass and max |u|
 *     at watchdog points.
 *
 * Conventions
 *   - Lattice units throughout. Masks are uint8 [nz][ny][nx], x fastest
 *     (flat index x + nx*(y + ny*z)), nonzero = solid. Flow is along +z.
 *   - Sites are the pore voxels in raster order (z slowest, x fastest), so
 *     the inlet sites are [0, a_in) and the outlet sites [n - a_out, n).
 *   - Host buffers are owned by the caller and only read or written during
 *     the call. Device memory is either caller-owned (flbm_bind_device_memory)
 *     or allocated by the library on first use and freed by flbm_destroy.
 *   - All device work is enqueued on the stream given to flbm_create (a
 *     hipStream_t; NULL means the null stream). Calls that return host data
 *     synchronise that stream.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Every call returns FLBM_OK (0) or a negative flbm_status; the text of
 *     the last error of a context is available from flbm_last_error.
 *   - Testing aids read from the environment at flbm_create: FLBM_NO_GRAPH=1
 *     launches every step directly instead of replaying captured graphs;
 *     FLBM_NO_BUF=1 takes the 64-bit addressing path of lattices past 4 GiB
 *     (no raw buffer instructions, no compact pull table) at any size.
 *   - Profiling: FLBM_PROFILE=1 at flbm_create puts a roctx range (recorded
 *     by rocprofv3 --marker-trace) around flbm_step, flbm_batch_step and
 *     every kernel launch of a step -- "flbm phase pass", "flbm colour step",
 *     "flbm stream-collide", "flbm step finalize", "flbm observables",
 *     "flbm controller" -- and launches steps directly instead of replaying
 *     graphs, so each kernel lies inside its range. The roctx library is
 *     opened at run time; without it the ranges are no-ops. Results are
 *     unchanged.
 */
#ifndef FLUXLBM_H
#define FLUXLBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t flbm_status;

#define FLBM_OK 0
#define FLBM_EINVAL (-1)    /* bad argument or parameter */
#define FLBM_ENOINLET (-2)  /* no pore site on the inlet plane: eq. potential divides by A = 0 */
#define FLBM_ENOMEM (-3)    /* host or device allocation failed */
#define FLBM_EHIP (-4)      /* HIP runtime error; text in flbm_last_error */
#define FLBM_EUNSTABLE (-5) /* watchdog saw a non-finite value or max|u| above the limit */
#define FLBM_EINDEX (-6)    /* 19 * padded sites does not fit a signed 32-bit index */
#define FLBM_EBOUND (-7)    /* caller's device buffer is smaller than flbm_device_bytes */
#define FLBM_ESTATE (-8)    /* call not valid in the context's current state */
#define FLBM_ESCRATCH (-9)  /* input larger than the allocation-free entry point's scratch holds */

/* Storage precision of the distributions. Boundary sums and the inlet
 * density are FP64 in every mode. */
#define FLBM_FP64 0
#define FLBM_FP32 1
#define FLBM_FP16DEV 2 /* FP16 storage of scaled deviations f - w_q, FP32 arithmetic (the colour
                          model keeps its D3Q7 colours and phase field in FP32) */

/* Collision model. */
#define FLBM_BGK 0
#define FLBM_COLOUR 1 /* two-fluid colour-gradient model (Appendix A) */
#define FLBM_MRT 2    /* single fluid, MRT collision of Appendix A (the paper's Sec. 3 runs) */

/* Treatment of the z faces. FLBM_Z_FLUX is the paper's set-up: flux inlet at
 * z = 0, pressure outlet at z = nz-1 (Methods, last paragraph). The other two
 * close the box (periodic, or bounce-back walls beyond both z faces). */
#define FLBM_Z_FLUX 0
#define FLBM_Z_PERIODIC 1
#define FLBM_Z_WALL 2

typedef struct flbm_params {
    int32_t nx, ny, nz;         /* mask dimensions; nz >= 3 */
    int32_t periodic_x;         /* 1: periodic in x; 0: bounce-back walls beyond x faces */
    int32_t periodic_y;         /* same for y */
    int32_t z_mode;             /* FLBM_Z_* */
    int32_t reservoir_layers;   /* z-planes forced to fluid at each end (pure-fluid reservoirs) */
    int32_t precision;          /* FLBM_FP64 / FLBM_FP32 / FLBM_FP16DEV */
    int32_t model;              /* FLBM_BGK / FLBM_COLOUR / FLBM_MRT */
    int32_t watchdog_every;     /* mass, max|u| and finiteness checked at least this often (steps) */
    double tau;                 /* relaxation time, > 1/2; nu = (tau - 1/2)/3 */
    double rho0;                /* reference density of the incompressible model (eq. m357) */
    double q_target;            /* target volumetric flux Q* through z = 0, lu^3/lt */
    double rho_out;             /* outlet density; pressure p = rho/3 (eq. pressure) */
    double alpha;               /* colour model: interfacial-stress strength (Appendix A) */
    double beta;                /* colour model: recolouring strength (Appendix A) */
    double phi_solid;           /* colour model: phase value seen at solid neighbours */
    double umax_limit;          /* watchdog threshold on |u| (the paper's rule of thumb: 0.1) */
} flbm_params;

typedef struct flbm_ctx flbm_ctx;

/* Fill *p with defaults: periodic x and y, FLBM_Z_FLUX, FP32, BGK, tau 0.8,
 * rho0 1, q_target 0, rho_out 1, watchdog every 1000 steps, umax_limit 0.1,
 * alpha 0.005, beta 0.7, phi_solid 0. Dimensions are set to zero. */
flbm_status flbm_default_params(flbm_params *p);

/* Build the sparse pore lattice from a host solid mask (uint8 [nz][ny][nx],
 * nonzero = solid; copied, not kept) and create a context whose device work
 * goes to `hip_stream` (hipStream_t or NULL). No device memory is touched
 * until flbm_bind_device_memory or the first call that needs it.
 * Errors: FLBM_EINVAL (null pointer, dims, tau <= 1/2, rho0 <= 0, unknown
 * mode), FLBM_ENOINLET (FLBM_Z_FLUX with no pore site at z = 0),
 * FLBM_EINDEX (lattice too large for 32-bit indices), FLBM_ENOMEM. */
flbm_status flbm_create(const uint8_t *solid_mask, const flbm_params *p, void *hip_stream,
                        flbm_ctx **out);

/* Release the context and, if the library allocated it, its device memory. */
flbm_status flbm_destroy(flbm_ctx *c);

/* Device bytes the context needs (distributions in two copies, the int32
 * pull table and its compact form, FP64 reduction scratch and history). */
flbm_status flbm_device_bytes(const flbm_ctx *c, size_t *bytes);

/* Use caller-owned device memory (e.g. a torch uint8 tensor) of at least
 * flbm_device_bytes bytes, 256-byte aligned; it must outlive the context.
 * Only valid before any device memory is in use (else FLBM_ESTATE).
 * Uploads the pull tables and sets the rest state rho = rho_out, u = 0.
 * Errors: FLBM_EBOUND if too small, FLBM_EINVAL if null or misaligned. */
flbm_status flbm_bind_device_memory(flbm_ctx *c, void *dev_ptr, size_t bytes);

/* Counts: pore sites, inlet pore sites (the area A of eq. potential), outlet
 * pore sites. */
flbm_status flbm_num_sites(const flbm_ctx *c, int64_t *n_sites, int64_t *a_in, int64_t *a_out);

/* Site coordinates, host int32 [n_sites][3] = (x, y, z), in site order. */
flbm_status flbm_get_site_coords(const flbm_ctx *c, int32_t *xyz);

/* Set every pore site to the equilibrium with density rho and velocity u
 * (App. B equilibrium), reset the step counter, history and watchdog flag. */
flbm_status flbm_init_equilibrium(flbm_ctx *c, double rho, double ux, double uy, double uz);

/* Target flux Q* (eq. flux) used from the next step on. */
flbm_status flbm_set_target_flux(flbm_ctx *c, double q_target);

/* Outlet density used from the next step on. */
flbm_status flbm_set_outlet_density(flbm_ctx *c, double rho_out);

/* Enqueue n time steps on the context's stream (asynchronous). Within the n
 * steps each step kernel also ends the step before it (history record,
 * carried inlet sum); the last one ends in a launch of its own (every step
 * does, for the colour model and under the learned controller), so once the
 * stream has reached the end of the call every step is recorded. */
flbm_status flbm_step(flbm_ctx *c, int32_t n);

/* Wait for the context's stream. Returns FLBM_EUNSTABLE if a watchdog check
 * since the last init/write found a non-finite value or |u| > umax_limit. */
flbm_status flbm_sync(flbm_ctx *c);

/* Boundary values of the last completed step (synchronises): Q_in (sum of
 * u_z over the inlet sites after the pressure condition; equals Q* up to
 * rounding), Q_out (the same sum over the outlet sites), rho_in (eq.
 * potential), rho_out. Any pointer may be NULL. */
flbm_status flbm_get_boundary(flbm_ctx *c, double *q_in, double *q_out, double *rho_in,
                              double *rho_out);

/* Per-step FP64 history of the last n steps, oldest first, 7 doubles per
 * step: rho_in, Q_in, Q_out, total mass, max|u|, sum N_A, sum N_B. Mass,
 * max|u| and the colour sums are NaN on steps that were not watchdog points
 * (the colour sums always for the single-fluid model). n must not exceed the
 * number of steps taken nor the ring capacity (flbm_history_capacity).
 * Synchronises. */
flbm_status flbm_get_history(flbm_ctx *c, double *buf, int32_t n);
flbm_status flbm_history_capacity(const flbm_ctx *c, int32_t *cap);

/* Number of steps taken since the last init/write. */
flbm_status flbm_step_count(const flbm_ctx *c, int64_t *steps);

/* Density and velocity of every pore site (host FP64 arrays of n_sites,
 * site order), from the stored post-collision state; collision conserves
 * them, so they are the post-boundary moments of the last step. Any pointer
 * may be NULL. Synchronises. */
flbm_status flbm_read_fields(flbm_ctx *c, double *rho, double *ux, double *uy, double *uz);

/* Read / write the stored distributions as host FP64 [19][n_sites] (q
 * slowest, site order; absolute values f_q, not deviations). Writing
 * converts to the storage precision, resets the step counter, history and
 * watchdog flag. Synchronise. */
flbm_status flbm_read_distributions(flbm_ctx *c, double *f);
flbm_status flbm_write_distributions(flbm_ctx *c, const double *f);

/* ---------------------------------------------------------------------
 * Learned inlet controller (a learned addition on top of the method: the
 * paper's plain update of eq. potential stays its fallback and judge).
 *
 * flbm_mlp is a 32 -> 128 -> 128 -> 1 multilayer perceptron with tanh
 * hidden layers whose products run on the matrix cores with BF16 operands
 * and FP32 accumulation; FP32 master weights, mean-squared-error loss, Adam.
 * Parameter order (FP32): W1 [128][32], b1 [128], W2 [128][128], b2 [128],
 * W3 [1][128], b3 [1] (flbm_mlp_num_params). Inputs are device FP32 arrays
 * [batch][32], targets and outputs device FP32 [batch]; work goes to the
 * stream given at creation. */
typedef struct flbm_mlp flbm_mlp;
flbm_status flbm_mlp_create(int32_t max_batch, void *hip_stream, flbm_mlp **out);
flbm_status flbm_mlp_destroy(flbm_mlp *m);
flbm_status flbm_mlp_num_params(int32_t *n);
/* host FP32 parameters; setting them also resets the optimiser state */
flbm_status flbm_mlp_set_params(flbm_mlp *m, const float *host, int32_t n);
flbm_status flbm_mlp_get_params(flbm_mlp *m, float *host, int32_t n);
flbm_status flbm_mlp_forward(flbm_mlp *m, const float *dev_x, float *dev_y, int32_t batch);
/* loss and its gradient with respect to every parameter (host FP32), for checks */
flbm_status flbm_mlp_gradients(flbm_mlp *m, const float *dev_x, const float *dev_t, int32_t batch,
                               float *host_grads, float *host_loss);
/* one Adam step (beta 0.9, 0.999, eps 1e-8) at learning rate lr; host_loss
 * may be NULL (then the call does not synchronise) */
flbm_status flbm_mlp_train_step(flbm_mlp *m, const float *dev_x, const float *dev_t, int32_t batch, float lr,
                                float *host_loss);
/* C = A B with A (M x K) element (i,k) at A[i*a_rs + k*a_cs], B (K x N)
 * element (k,j) at B[k*b_rs + j*b_cs], C[i*c_rs + j]; FP32 arrays on the
 * device, operands rounded to BF16, FP32 accumulation (the network's matrix
 * core routine, exposed for testing). Asynchronous on hip_stream. */
flbm_status flbm_gemm_bf16(const float *A, int64_t a_rs, int64_t a_cs, const float *B, int64_t b_rs,
                           int64_t b_cs, float *C, int64_t c_rs, int32_t M, int32_t N, int32_t K,
                           void *hip_stream);

typedef struct flbm_controller_params {
    float geometry[15];   /* static inputs 0..14 of the network (sample and inlet-slice statistics) */
    float margin;         /* >= 0: the proposal aims below the prediction, r - margin */
    double drho_ref;      /* reference inlet-outlet density difference (input 31, absolute proposal) */
    double gain;          /* fraction of the step from the plain density to the proposal taken */
    double trust0;        /* initial bound on |Q_in - Q*| / Q* that a proposal may cause */
    double release_tol;   /* period-mean |Q_out - Q*| / Q* that returns control to the
                             plain update for good */
    int32_t trust_decisions; /* the bound decays linearly to zero over this many decisions */
    int32_t relative;     /* 0: r = log(drho_inf / drho_ref); 1: r = log(drho_inf / drho) */
    int32_t stall_decisions; /* > 0: release when the outlet error has not improved by 10 %
                                over this many decisions */
    int32_t period;       /* steps per decision (>= 1; even values average the period-two
                             oscillation of the outlet flux) */
} flbm_controller_params;

/* Attach (net != NULL) or detach (net == NULL) the controller. While
 * attached, it sums the outlet flux over periods of `period` steps and takes
 * a decision at the end of each period. The network reads 32 inputs: the 15
 * geometry values, the errors (Qbar - Q*) / |Q*| clipped to [-2, 2] of the
 * period-mean outlet flux Qbar at lags 1, 2, 3, 4, 6, 8, 11, 16, 22, 32, 45,
 * 64, 90, 128, 180, 250 periods back (0 before the first step), and
 * log10(drho / drho_ref) / 3 clipped to [-1, 1] (-1 if drho <= 0), drho =
 * rho_in - rho_out of the last step. Its output r is the predicted steady
 * density difference drho_inf, either absolute (relative = 0: r =
 * log(drho_inf / drho_ref) clipped to [-4, 4], proposal rho_hat = rho_out +
 * drho_ref exp(r)) or as the remaining relative rise (relative = 1: r =
 * log(drho_inf / drho) clipped to [-2, 3], rho_hat = rho_out + drho exp(r)),
 * with r replaced by r - margin (an undershoot that leaves the last part of
 * the rise to the plain update).
 * The proposal is held for the next period; every step in it uses
 *   rho_in = rho_plain + clip(gain (rho_hat - rho_plain), +-bound rho0 |Q*| / A)
 * with rho_plain the update of eq. potential of that step and bound = trust0
 * (1 - n / trust_decisions)^+ after n decisions, i.e. |Q_in - Q*| / Q* <=
 * bound. No proposal once the period-mean outlet error has met release_tol
 * (after two periods), or (stall_decisions > 0) once it has not fallen below
 * 0.9 times its best value for stall_decisions decisions (both for good),
 * when Q* <= 0, when relative and drho <= 0, or when the network output or
 * the proposal is not finite. With trust0 = 0 the run is the plain method
 * exactly (the inputs are still recorded). The network must outlive the
 * attachment. Flux mode only (else FLBM_ESTATE). Synchronises. */
flbm_status flbm_set_controller(flbm_ctx *c, const flbm_mlp *net, const flbm_controller_params *p);
/* The controller's last n decisions, oldest first (n <= flbm_history_capacity
 * and n <= the decisions taken since the attachment): inputs x[n][32] (FP32)
 * and aux[n][4] = {drho, rho_plain, r, offset at the decision step} (FP64).
 * Synchronises. */
flbm_status flbm_controller_trace(flbm_ctx *c, int32_t n, float *x, double *aux);

/* Inlet density override (a hook for a caller-side controller): while set,
 * every step uses rho_in = rho_plain + clip(*rho_in_or_null - rho_plain,
 * +-trust rho0 |Q*| / A), i.e. the plain update of eq. potential still
 * judges it: |Q_in - Q*| / |Q*| <= trust (Q* at the time of the call).
 * NULL clears it. It takes precedence over an attached controller's proposal.
 * Flux mode only (else FLBM_ESTATE); a non-finite density or a negative
 * trust is FLBM_EINVAL. Synchronises; survives steps, not a re-initialisation. */
flbm_status flbm_set_inlet_density_override(flbm_ctx *c, const double *rho_in_or_null, double trust);
/* attached flag, released flag, offset at the last decision, decisions taken
 * (synchronises) */
flbm_status flbm_controller_state(flbm_ctx *c, int32_t *active, int32_t *released, double *delta,
                                  int64_t *decisions);

/* ---------------------------------------------------------------------
 * Batched stepping: many lattices (porous samples of uneven size, each with
 * its own target flux, outlet density and state) advanced together by ONE
 * kernel launch per step. The launch walks a work list of (sample, tile
 * range) items with a persistent grid; each sample's step is exactly what
 * flbm_step would do (the same tile work, its own inlet sum of eq. potential
 * in FP64, its own history and watchdog). Runs of `chunk` steps are captured
 * as a HIP graph and replayed.
 *
 * The samples are ordinary contexts with device memory bound, all on the
 * same device and stream, of one precision and one single-fluid model
 * (FLBM_BGK or FLBM_MRT; else FLBM_EINVAL), no controller attached and not
 * the colour model (FLBM_ESTATE). They stay usable on their own (init,
 * targets, reads, flbm_step) and must outlive the batch. */
typedef struct flbm_batch flbm_batch;

#define FLBM_ORDER_SAMPLE 0     /* the items of one sample after another */
#define FLBM_ORDER_INTERLEAVE 1 /* round robin over the samples */
#define FLBM_ORDER_LARGEST 2    /* round robin, largest samples first */

typedef struct flbm_schedule {
    int32_t grid;           /* blocks of the persistent launch; 0: one block per work item */
    int32_t order;          /* FLBM_ORDER_* */
    int32_t tiles_per_item; /* consecutive tiles of one sample per work item (>= 1) */
    int32_t chunk;          /* steps per captured graph (>= 1; graphs are used when even) */
    int32_t occupancy;      /* 0: the compiler's register budget; 8: at most 64 VGPRs (8 waves per
                               SIMD) for the steps that record no observables; only for grid 0
                               with one tile per item, and only where that kernel needs no
                               scratch (else the compiler's budget is used) */
} flbm_schedule;

/* samples: n context pointers (not copied beyond the call's lifetime of the
 * array; the contexts themselves must outlive the batch). Default schedule:
 * one block per item, interleaved, 4 tiles per item, chunk 64, compiler budget. */
flbm_status flbm_batch_create(int32_t n, flbm_ctx *const *samples, flbm_batch **out);
flbm_status flbm_batch_destroy(flbm_batch *b);
flbm_status flbm_batch_set_schedule(flbm_batch *b, const flbm_schedule *s);
flbm_status flbm_batch_get_schedule(const flbm_batch *b, flbm_schedule *s);
/* n steps of every sample, asynchronous on the samples' stream */
flbm_status flbm_batch_step(flbm_batch *b, int32_t n);
/* synchronise; FLBM_EUNSTABLE if a sample's watchdog tripped (its index in
 * *first_unstable, else -1) */
flbm_status flbm_batch_sync(flbm_batch *b, int32_t *first_unstable);
/* n steps launched one by one (no graph, no watchdog) between two HIP events
 * on the samples' stream: the mean duration of one batched launch */
flbm_status flbm_batch_time(flbm_batch *b, int32_t n, double *ms_per_step);
/* Choose the schedule (persistent grid 0 / 2 / 4 / 8 / 16 blocks per compute
 * unit, the three orders, 1 / 4 / 16 tiles per item) by timing trial_steps
 * launches of each, with both register budgets for one block per single-tile
 * item (1 + trial_steps steps of every sample per candidate: the samples
 * advance), or take it from cache_path (text lines "v2 arch precision model
 * pull_formats log2(sites) grid order tiles_per_item occupancy ms", with
 * pull_formats a bit mask of the pull-table formats the samples read: 1 the
 * int32 table, 2 16-bit codes, 4 compact codes, 8 run codes; lines without the "v2" tag
 * are ignored; NULL: no cache), where a new choice is appended. The chosen
 * schedule is set. */
flbm_status flbm_batch_autotune(flbm_batch *b, const char *cache_path, int32_t trial_steps, flbm_schedule *best,
                                double *best_ms);
const char *flbm_batch_last_error(const flbm_batch *b);

/* Two-fluid colour model (Appendix A; FLBM_COLOUR contexts only, else
 * FLBM_ESTATE). The colours A (non-wetting) and B (wetting) are D3Q7
 * distributions over the velocities q = 0..6 with weights 1/3, 1/9.
 *
 * flbm_init_colour: momentum at rest (rho = 1, u = 0) and A_q = w_q na[s],
 *   B_q = w_q nb[s] from host FP64 arrays of n_sites colour densities; resets
 *   the step counter, history and watchdog flag.
 * flbm_read_colour / flbm_write_colour: host FP64 [7][n_sites] each, site
 *   order; writing resets the step counter.
 * flbm_read_phase: phi = (N_A - N_B)/(N_A + N_B) of the stored state, host
 *   FP64 [n_sites].
 * All synchronise. */
flbm_status flbm_init_colour(flbm_ctx *c, const double *na, const double *nb);
flbm_status flbm_read_colour(flbm_ctx *c, double *A, double *B);
flbm_status flbm_write_colour(flbm_ctx *c, const double *A, const double *B);
flbm_status flbm_read_phase(flbm_ctx *c, double *phi);

/* Host copy of the pull table, int32 [18][n_sites] (row q-1 for direction
 * q = 1..18): the flat index into a [19][n_pad] distribution array that
 * streams into (q, site) -- q*n_pad + source site, opp(q)*n_pad + site for
 * halfway bounce-back, or 19*n_pad for a boundary unknown (the unknowns of
 * Methods, before eq. inlet). Host-only; needs no device. */
flbm_status flbm_get_pull_table(const flbm_ctx *c, int32_t *nbr);

/* Pull-table format of the single-fluid step (Methods: streaming pulls each
 * population from the site x - xi_q; the table only says where that value
 * is stored). Every format addresses the same slots, so results are bitwise
 * equal; they differ in the bytes a step reads per site.
 *   FLBM_PULL_INT32    the int32 table above: 72 bytes per site.
 *   FLBM_PULL_HALF     per tile of 512 consecutive sites one int32 base per
 *                      direction, per site 16-bit codes, two to a word:
 *                      code c <= 0xFFFD is the flat index base + c, 0xFFFE
 *                      the boundary-unknown sentinel, 0xFFFF the bounce-back
 *                      slot opp(q)*n_pad + site: 36 bytes per site.
 *   FLBM_PULL_COMPACT  as HALF, but a tile whose sources fit takes 8-bit
 *                      codes against the site's position p in the tile:
 *                      c <= 0xFD is base + p + c, 0xFE the sentinel, 0xFF
 *                      bounce-back: 18 bytes per site.
 *   FLBM_PULL_RUN      (the default where available) as COMPACT, but the
 *                      step (the colour model's second pass) reads the
 *                      8-bit codes of a tile as run codes where it has
 *                      them: per wave of 64 sites, a per-site mask of the
 *                      directions whose code differs from the previous
 *                      site's and the wave's list of those codes (at most
 *                      512): 8 bytes per site, 12 where a wave lists more
 *                      than 256 codes. Not in the colour model's FP16
 *                      step, which reads the 8-bit codes (decoding runs
 *                      costs it more than the bytes saved). COMPACT and RUN
 *                      share one table, so switching between them rebuilds
 *                      nothing.
 * A tile whose sources of some direction span more than a form's range
 * falls back to the next wider form, down to the int32 table. Both passes of
 * the colour model read it too (the phase pass directions 1..6). Lattices
 * too large for the 4 GiB buffer path have no compact table (FLBM_ESTATE for
 * the coded formats). limit16 (<= 0xFFFD) and limit8
 * (<= 0xFD) below the defaults (0 means the default) are a testing aid that
 * sends more tiles to the wider forms. Synchronises; rebuilds the codes on
 * the host (O(18 n)) when a limit changes. */
#define FLBM_PULL_INT32 0
#define FLBM_PULL_HALF 1
#define FLBM_PULL_COMPACT 2
#define FLBM_PULL_RUN 3
flbm_status flbm_set_pull_format(flbm_ctx *c, int32_t format, int32_t limit16, int32_t limit8);
/* The format in use and, of the `tiles` tiles, how many read 8-bit and
 * 16-bit codes (the rest read the int32 table; both 0 for FLBM_PULL_INT32).
 * Host-only. */
flbm_status flbm_pull_format_info(const flbm_ctx *c, int32_t *format, int64_t *tiles8, int64_t *tiles16,
                                  int64_t *tiles);
/* Host copy of the compact table: 16-bit codes uint32 [9][n_pad] (word k:
 * direction 2k+1 in bits 0-15, 2k+2 in bits 16-31), 8-bit codes uint32
 * [4][n_pad] (byte j of word k: direction 4k+j+1) and uint16 [n_pad]
 * (directions 17 in bits 0-7, 18 in bits 8-15), and the header int32
 * [tiles][20] (entries 0..17: the base of direction q at q-1; entry 18 the
 * tile's form: 0 int32 table, 1 16-bit, 2 8-bit; entry 19: 1 if the 8-bit
 * tile also has run codes, else 0). A tile's rows in the forms it does not
 * use are zero. Any pointer may be NULL. Host-only; FLBM_ESTATE without a
 * compact table. */
flbm_status flbm_get_compact_pull(const flbm_ctx *c, uint32_t *codes16, uint32_t *codes8, uint16_t *codes8_tail,
                                  int32_t *hdr);
/* Of the 8-bit tiles, how many have run codes, and how many of their waves
 * list more than 256 codes (12 bytes per site instead of 8). Host-only. */
flbm_status flbm_pull_run_info(const flbm_ctx *c, int64_t *tiles_run, int64_t *waves_wide);
/* Host copy of the run codes: uint32 [n_pad][2] (word 0: bit q-1 set where
 * direction q's 8-bit code differs from the previous site's, always at a
 * wave's first site (sites 64w); bit 31 set on every site of a wave whose
 * list is longer than 256 bytes; word 1 of site 64w + l: bytes 4l..4l+3 of
 * the wave's list, the listed codes direction by direction in site order)
 * and uint32 [n_pad] (site 64w + l: bytes 256+4l..256+4l+3). Site 64w + l's
 * code of direction q is list entry off + r, off the listed codes of the
 * directions before q and r the listed codes of q at sites 64w..64w+l,
 * minus one. Zero in tiles without run codes. Any pointer may be NULL.
 * Host-only; FLBM_ESTATE without a compact table. */
flbm_status flbm_get_pull_runs(const flbm_ctx *c, uint32_t *runs, uint32_t *runs_hi);

/* Raw checkpoint of the stored state: flbm_state_bytes gives the size; save
 * copies the current distribution buffers (storage precision: f as
 * deviations, then A and B for the colour model), the step count and the
 * carried inlet sum to host memory; load restores them, so that a resumed
 * run is bitwise identical to an uninterrupted one. Synchronise. */
flbm_status flbm_state_bytes(const flbm_ctx *c, size_t *bytes);
flbm_status flbm_save_state(flbm_ctx *c, void *host, size_t bytes);
flbm_status flbm_load_state(flbm_ctx *c, const void *host, size_t bytes);

/* Testing aid: enabled = 0 turns collision off (relaxation rate 0), so a
 * step is pure streaming plus boundary conditions. */
flbm_status flbm_debug_set_collision(flbm_ctx *c, int32_t enabled);

/* Total mass, max |u| and a non-finite flag of the current state, computed
 * on the device from the stored distributions (synchronises). */
flbm_status flbm_get_observables(flbm_ctx *c, double *mass, double *umax, int32_t *nonfinite);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * observables of flbm_get_observables -- total mass sum_s rho_s, max |u|
 * (NaN if any value is not finite) and a non-finite flag -- of a state the
 * caller holds on the device, without a context and without allocating.
 *   f_dev      device distributions [19][n_pad] of the storage precision as
 *              deviations f - w_q (the layout flbm_device_layout gives);
 *              only read. Sites n_sites..n_pad-1 must hold zero deviations.
 *   precision  FLBM_FP64 / FLBM_FP32 / FLBM_FP16DEV (scaled deviations)
 *   n_sites    pore sites (mass counts rho - 1 over n_pad sites, plus n_sites)
 *   n_pad      padded site count, a multiple of 256, at most 67,108,864
 *              (FLBM_ESCRATCH beyond: the partial sums of its 256-site
 *              blocks live in a fixed device array of the library, about
 *              4 MiB per GPU, held until the process ends)
 *   rho0       reference density (u = j / rho0)
 *   hip_stream the work is enqueued there and the call synchronises it
 *   mass, umax, nonfinite  host outputs, any may be NULL
 * No device memory is allocated: the library's array is located once per
 * device (on the first call with that device current). Every call on a GPU
 * shares that GPU's array and rewrites the parts it reads, so calls that
 * overlap on one GPU (other threads or streams) race and must be serialised
 * by the caller. Errors: FLBM_EINVAL (null f_dev, n_sites outside [0,
 * n_pad], n_pad not a positive multiple of 256, rho0 <= 0, unknown
 * precision), FLBM_ESCRATCH, FLBM_EHIP. */
flbm_status flbm_state_observables_noalloc(const void *f_dev, int32_t precision, int64_t n_sites, int64_t n_pad,
                                           double rho0, void *hip_stream, double *mass, double *umax,
                                           int32_t *nonfinite);

/* Device pointers of the current distribution buffer (layout [19][n_pad] of
 * the storage type, deviations f - w_q) and of the pull table (int32
 * [18][n_pad]); for profiling and zero-copy inspection. */
flbm_status flbm_device_layout(const flbm_ctx *c, void **f_cur, void **nbr, int64_t *n_pad);

/* Profiling: recompute the inlet consistency sum from the state with the
 * inlet-plane reduction kernel, then run n steps launched one by one (no
 * graph, no watchdog reduction), each kernel bracketed by HIP events on the
 * context's stream; return the duration in milliseconds of the plane
 * reduction and the mean duration of the fused stream-collide kernel. (In a
 * run of steps the plane reduction runs only once: each step kernel carries
 * the next step's inlet sum.) For the colour model the step duration covers
 * both launches of a step (phase pass and colour step). The steps are real
 * steps. Synchronises. */
flbm_status flbm_profile_kernels(flbm_ctx *c, int32_t n, double *ms_plane, double *ms_step);

/* Stream-copy calibration kernel: copies `bytes` (a multiple of 16, both
 * pointers 16-byte aligned) from src to dst on `hip_stream`, 16 bytes per
 * lane with non-temporal loads and stores. For measuring attainable HBM
 * bandwidth beside the step. */
flbm_status flbm_copy_kernel(const void *src, void *dst, size_t bytes, void *hip_stream);

const char *flbm_status_string(flbm_status s);
const char *flbm_last_error(const flbm_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* FLUXLBM_H */
