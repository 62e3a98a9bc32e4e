/*
 * atns.h -- C ABI of the asynchrony-tolerant (AT) compressible-flow
 * right-hand-side library for AMD MI355X (gfx950).
 *
 * The library advances the compressible Euler / Navier-Stokes equations
 * (Sec. 2, Eq. 1 and App. A of arXiv 2506.03027) on a uniform periodic
 * Cartesian grid with the explicit fourth-order central difference (Eq. 2,
 * CD4 of App. B), or, for the second-order method of Table 1 cases 1-3
 * (rk = ATNS_LSERK2), with CD2 and the AT2 schemes.  The grid is split into a tensor product of blocks -- the
 * processing elements (PEs) of Sec. 3 -- that all live on one GPU.  Each
 * block reads the points it does not own (its halo, the "buffer points" of
 * Sec. 3) either synchronously (SA, Alg. 1) or from a ring of delayed time
 * levels, as the communication-avoiding (CAA, Alg. 2) or the
 * synchronization-avoiding (SAA, Alg. 3) algorithm would deliver them, with
 * the asynchrony-tolerant buffer extrapolation and updates of Sec. 3.1-3.2
 * (Eqs. 7-15, App. C) or with plain stale data (AS).
 *
 * Conventions
 * -----------
 * - Every function returns an atns_status; no function throws or aborts.
 *   ATNS_EINVAL reports a bad argument or configuration, ATNS_EHIP a failed
 *   HIP runtime call, ATNS_ENOMEM a failed device allocation, ATNS_ESTATE a
 *   call in the wrong state (e.g. stepping before a state is set).
 *   atns_last_error() returns a message for the last failure on a context.
 * - The library owns every device allocation it makes and frees it in
 *   atns_destroy().  Pointers passed in by the caller are borrowed for the
 *   duration of the call only.
 * - "dev" pointers are device (HIP) pointers on the context's device;
 *   "host" pointers are ordinary host memory.
 * - Field layout: structure of arrays, 5 conserved variables
 *   (rho, rho u, rho v, rho w, rho E_t), each a contiguous [nz][ny][nx]
 *   array with x fastest: element (v, k, j, i) at ((v*nz + k)*ny + j)*nx + i.
 *   The element type is float (ATNS_F32) or double (ATNS_F64).
 * - Work is enqueued on the stream given to atns_create() (NULL = the null
 *   stream).  Only atns_reduce(), atns_get_state(on_host=1),
 *   atns_get_delays(), atns_checkpoint() and atns_restore() synchronize
 *   with the host.
 * - Steps are numbered n = 0, 1, ...; step n advances U^n to U^{n+1}.
 *
 * Neighbour slots (index into delay arrays):
 *   0 -x   1 +x   2 -y   3 +y   4 -z   5 +z
 *   6 (-x,-y)  7 (+x,-y)  8 (-x,+y)  9 (+x,+y)
 *  10 (-x,-z) 11 (+x,-z) 12 (-x,+z) 13 (+x,+z)
 *  14 (-y,-z) 15 (+y,-z) 16 (-y,+z) 17 (+y,+z)
 * Euler uses the six faces (halo depth 2).  Navier-Stokes uses faces of
 * depth 4 (5 with the filter on) and the twelve 2x2 edge regions (viscous
 * terms as repeated first derivatives).  Delays are int8 arrays
 * [nblocks][ATNS_NSLOTS].
 */
#ifndef ATNS_H
#define ATNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ATNS_NSLOTS 18
#define ATNS_NDIAG 7

typedef struct atns_ctx atns_ctx;

typedef enum {
  ATNS_OK = 0,
  ATNS_EINVAL = -1,
  ATNS_ENOMEM = -2,
  ATNS_EHIP = -3,
  ATNS_ESTATE = -4,
  ATNS_ENONFINITE = -5
} atns_status;

enum { ATNS_EULER = 0, ATNS_NS = 1 };                 /* physics          */
enum { ATNS_RK4 = 0, ATNS_LSERK4 = 1, ATNS_LSERK2 = 2 }; /* time integrator */
enum { ATNS_SA = 0, ATNS_AS = 1, ATNS_AT = 2 };       /* halo treatment   */
enum { ATNS_CAA = 0, ATNS_SAA = 1 };                  /* delay algorithm  */
enum { ATNS_F32 = 0, ATNS_F64 = 1 };                  /* state precision  */

typedef struct {
  int32_t ndim;          /* 2 or 3; ndim == 2 requires n[2] == 1, nblk[2] == 1 */
  int32_t n[3];          /* global points nx, ny, nz                          */
  double len[3];         /* periodic box lengths; h_d = len[d] / n[d]         */
  int32_t nblk[3];       /* blocks per direction                              */
  const int32_t* split[3]; /* optional host arrays of nblk[d] block sizes
                              summing to n[d]; NULL = even split (the first
                              n % nblk blocks get one extra point)            */
  int32_t physics;       /* ATNS_EULER | ATNS_NS                              */
  double gamma, mach, re, pr; /* gas: p = (gamma-1)(rho E - rho|u|^2/2),
                              T = gamma M^2 p / rho, mu = 1,
                              kappa = 1/((gamma-1) M^2 Pr); re, pr NS only    */
  int32_t rk;            /* ATNS_RK4 | ATNS_LSERK4 (Eq. 3, Table 4): CD4 and
                            AT4 (C = 5 delayed levels).  ATNS_LSERK2 (App. B,
                            A = {0, -1/2}, B = {1/2, 1}): the second-order
                            method of Table 1 cases 1-3, CD2 (App. B, a = 1,
                            b = 0) in the interior and AT2 (C = 3 levels,
                            Eq. 14 and App. C) at block boundaries; the halo
                            depth stays that of CD4 (the outer layer is read
                            with weight 0).  The learned halo needs C = 5.   */
  int32_t mode;          /* ATNS_SA | ATNS_AS | ATNS_AT                       */
  int32_t algo;          /* ATNS_CAA | ATNS_SAA                               */
  int32_t L;             /* delay bound: delays are 0..L-1 (Alg. 2, 3)        */
  uint64_t seed;         /* SAA delay stream seed                             */
  int32_t precision;     /* ATNS_F32 | ATNS_F64                               */
  int32_t filter;        /* 0: off.  1: tenth-order Pade low-pass filter of
                            the conserved variables after every step (Sec. 2;
                            Sec. 5.2 uses it with alpha_f = 0.499), applied
                            block by block, x then y then z, with the halo
                            depth raised to 5 (see atns_filter_state).
                            Navier-Stokes contexts only; not with batches,
                            atns_step_async or the learned halo.           */
  double filter_alpha;   /* alpha_f, -0.5 < alpha_f <= 0.5 (0.5: identity)  */
} atns_config;

/* Library version string (static storage). */
const char* atns_version(void);

/* Create a context on the current HIP device.  Validates the configuration
 * (EINVAL: block smaller than the halo depth in an active direction, split
 * not summing to n, L < 1 or L > 16, unknown enums, ndim == 2 with nz != 1,
 * a Navier-Stokes grid with 5 nx ny nz >= 2^31 points; with the filter on:
 * Euler physics, alpha_f outside (-0.5, 0.5], or a block longer than 256
 * points along an active axis)
 * before any device call.  stream: a hipStream_t, or NULL.  On success *out
 * owns all device buffers: state and RK registers, the delayed-level ring
 * (C + 2L - 1 levels of each block's boundary layers in modes AT and AS,
 * C + L in SA with L > 1; C = 5 for AT4, 3 for AT2) and tables. */
atns_status atns_create(const atns_config* cfg, void* stream, atns_ctx** out);

/* Free every resource of the context.  NULL is accepted. */
atns_status atns_destroy(atns_ctx* ctx);

/* Message of the last failure on ctx (never NULL). */
const char* atns_last_error(const atns_ctx* ctx);

/* Set U^step := dev_U (borrowed device array in the field layout) and make
 * `step` the current step.  The state is also recorded as history level
 * `step` (its boundary layers go into ring slot step mod D), so calling this
 * for consecutive steps m0..m1 builds a delayed history ending at m1. */
atns_status atns_set_state(atns_ctx* ctx, const void* dev_U, int64_t step);

/* Copy the current state into dst (device pointer if on_host == 0, host
 * pointer otherwise; host copies synchronize). */
atns_status atns_get_state(const atns_ctx* ctx, void* dst, int32_t on_host);

/* Analytic initial field, evaluated in FP64 on the device and rounded to the
 * context precision, set as U^step exactly as atns_set_state would (ring
 * slot included).  Coordinates x_i = i len/n (periodic, no duplicated end).
 *  ATNS_CASE_VORTEX: the isentropic vortex used for the inviscid tests
 *    (Sec. 5.1 tests the method on a vortex; this is the textbook translating
 *    isentropic vortex): rho_inf = p_inf = T_inf = 1, p = rho T, freestream
 *    of speed mach*sqrt(gamma) along (1,1)/sqrt2 (2-D) or (1,1,1)/sqrt3
 *    (3-D, vortex axis z); perturbation du = -(beta/2pi)(y-yc) e^((1-r^2)/2),
 *    dv = (beta/2pi)(x-xc) e^((1-r^2)/2), T = 1 - (gamma-1) beta^2 e^(1-r^2)
 *    / (8 gamma pi^2), rho = T^(1/(gamma-1)), r the minimum-image distance to
 *    the centre carried by the freestream for time t.  params (np <= 5, in
 *    this order, defaults in brackets): t [0], beta [5], mach [0.5],
 *    xc [5], yc [5].
 *  ATNS_CASE_TGV: the Taylor-Green vortex of Sec. 5.2 (Eq. 16) with
 *    rho0 = U0 = L0 = 1, v = -cos x sin y cos z (the divergence-free sign),
 *    uniform T0 = 1 so rho = gamma M^2 p, M = cfg.mach; 3-D only; np = 0.
 * EINVAL for unknown cases or bad parameter lists. */
enum { ATNS_CASE_VORTEX = 0, ATNS_CASE_TGV = 1 };
atns_status atns_init_case(atns_ctx* ctx, int32_t case_id, const double* params, int32_t np, int64_t step);

/* Checkpoint and restart.  atns_checkpoint with host_blob == NULL stores the
 * record size in *bytes; otherwise it writes the restart record into the
 * host buffer host_blob of *bytes bytes (EINVAL if smaller than the record,
 * ESTATE before any state is set), sets *bytes to the record size and
 * synchronizes.  The record holds the state, the delayed-level ring, the
 * step number, dt and a fingerprint of the configuration (grid, blocks,
 * physics, scheme, delays, seed, precision).  atns_restore accepts only a
 * record of an identically configured context (EINVAL otherwise, nothing
 * changed) and leaves the context as the checkpointed one was, so stepping
 * on gives the same bits.  Learned-halo parameters and settings are not
 * part of the record (atns_mlp_get_params / atns_mlp_set_params). */
atns_status atns_checkpoint(atns_ctx* ctx, void* host_blob, size_t* bytes);
atns_status atns_restore(atns_ctx* ctx, const void* host_blob, size_t bytes);

/* Current step number n. */
atns_status atns_get_step(const atns_ctx* ctx, int64_t* step);

/* Fixed time step (dt > 0).  The AT weights assume a constant dt (Sec. 3.1). */
atns_status atns_set_dt(atns_ctx* ctx, double dt);

/* Inject delays for steps step0 .. step0+nsteps-1 (host int8 array
 * [nsteps][nblocks][ATNS_NSLOTS]); they replace the CAA/SAA draws for those
 * steps.  The guard of Alg. 3 still applies: a delay above L-1, or one that
 * needs a level older than the history (k > n - C + 1), becomes 0.  nsteps
 * == 0 clears all injected delays. */
atns_status atns_set_delays(atns_ctx* ctx, int64_t step0, int32_t nsteps, const int8_t* host_k);

/* The delays (after the guard) that step `step` uses, into a host int8
 * array [nblocks][ATNS_NSLOTS].  Synchronous steps (SA mode, or step < C)
 * report all zeros and set *synchronous = 1. */
atns_status atns_get_delays(atns_ctx* ctx, int64_t step, int8_t* host_k, int32_t* synchronous);

/* Right-hand side R(U^n) of the current state, into dev_R (field layout,
 * context precision), with the halo values that stage `stage` of the current
 * step reads (0 <= stage < s; s = 4 for RK4, 5 for LSERK4, 2 for LSERK2):
 * under AT the buffer extrapolation of Eqs. 14-15 for stage 0 and the
 * RK-consistent buffer update of Eqs. 8-13 (Table 5, App. C) for later
 * stages, Uhat^(e) = sum_l W[e][k][l] U^{n-k-l}; under AS the stale level
 * U^{n-k} for every stage; synchronous steps (SA mode, or n < C) read the
 * current state itself, whatever the stage.  The owned points always take
 * the current state, so this evaluates the stage operator of Eq. 1 on U^n
 * with that stage's halo.  Does not advance the step.  EINVAL for a stage
 * outside 0..s-1 or a null pointer; ESTATE before a state is set. */
atns_status atns_rhs(atns_ctx* ctx, int32_t stage, void* dev_R);

/* Advance nsteps steps (asynchronous on the context stream).  Each step: the
 * delay draw, s fused stencil + RK-stage kernels (the halo of stage e from
 * the ring with the FP64 weights W[e][k][:]), and the ring write of U^{n+1}
 * in the last stage.  With the filter on, the last stage leaves U^{n+1}
 * unfiltered, the three filter passes of atns_filter_state follow (halos of
 * the step's kind: synchronous steps read the neighbours' current values of
 * each pass input, AT steps the neighbours' level n+1 extrapolated from the
 * C delayed levels with the Lagrange weights of Eqs. 14-15 at delay k+1, AS
 * steps the newest delayed level), and the filtered field's boundary layers
 * go into the ring (for steps with delayed halos in one launch, see
 * atns_set_filter_fusion). */
atns_status atns_rk_step(atns_ctx* ctx, int32_t nsteps);

/* Compensated classical RK4 steps (on != 0).  The accumulator then holds
 * only the step's increments, and the last stage forms U^{n+1} = U^n +
 * (increments + c) with Knuth's TwoSum, keeping the sum's rounding error c
 * per point and variable for the next step (a device array the size of the
 * state, allocated on the first call).  Single-precision state so carries
 * the time integration to about twice its precision, at the cost of reading
 * U^n and reading and writing c in the last stage.  c is cleared whenever a
 * state is set (atns_set_state, atns_init_case, atns_restore); checkpoints
 * do not hold it.  EINVAL for other integrators, with the filter, and later
 * in atns_step_async.  Default off. */
atns_status atns_set_compensation(atns_ctx* ctx, int32_t on);

/* Apply the configured filter (Sec. 2; a reading, since the paper does not
 * define it across PEs) to the current state in place, with synchronous
 * halos, and rewrite the ring slot of the current step.  Along each axis in
 * turn, every block solves
 *   alpha f^[i-1] + f^[i] + alpha f^[i+1] = sum_{m=0..5} (a_m/2)(f[i+m] + f[i-m])
 * on its own n points of each grid line, i = 0..n-1, the a_m fixed by
 * T(pi) = 0 and tenth-order accuracy; the filtered values at i = -1 and
 * i = n are replaced by the halo values there, so each block solves alone.
 * The right-hand side reads five halo points beyond each face.  Arithmetic in
 * FP64, result rounded to the state precision.  EINVAL when the context has
 * no filter; ESTATE before a state is set.  Asynchronous on the context
 * stream. */
atns_status atns_filter_state(atns_ctx* ctx);

/* The six right-hand-side coefficients a_0..a_5 of the tenth-order filter
 * for alpha (host computation, no device).  EINVAL for alpha outside
 * (-0.5, 0.5] or a null pointer. */
atns_status atns_host_filter_coefficients(double alpha, double* a6);

/* Fused RK4 stage pairs (on != 0): 3-D Euler contexts with classical RK4 in
 * single precision run stages 1-2 and stages 3-4 as two kernels instead of
 * four.  Stage A of a pair is evaluated on the tile and a 2-point apron and
 * stage B follows in the same pass, so the intermediate stage field and the
 * first RK register update never go through HBM; this is possible because
 * asynchronous halos of every stage come from the delayed levels, not from
 * the neighbours' current stage (and under synchronous halos the apron is
 * computed from the global field).  Results are the same bits as the
 * separate stage kernels.  Other contexts, and tile shapes the pair kernel
 * is not built for (it takes (16,16), (32,8), (16,8), (32,16)), keep the
 * separate kernels.  Default off. */
atns_status atns_set_fusion(atns_ctx* ctx, int32_t on);

/* Halo assembly inside the first stage (on != 0; default off): in
 * graph-captured asynchronous steps of Euler contexts, the first stage
 * kernel computes, before its plane loop, the values of every stage at the
 * halo points its tile reads -- Eq. 7 with Eqs. 8-15 (AT) or the stale level
 * (AS), from the ring levels and the step's delays, which it draws itself --
 * and writes them for the later stages, in place of a separate halo kernel
 * launch.  Same arithmetic, so the same bits either way.  Not applied to
 * Navier-Stokes contexts, batch members, steps with the learned halo or the
 * fused stage pairs, or eager steps.  It saves a launch and one halo write
 * and read, but the tile's assembly phase before its plane loop is
 * latency-bound, and on the vortex workloads the step is 1-2% slower.
 * Errors: ATNS_EINVAL for a null context. */
atns_status atns_set_halo_fusion(atns_ctx* ctx, int32_t on);

/* The filter of a step with delayed halos (AT or AS, step >= C) in one
 * launch (on != 0; default on): with delayed halos no filter pass reads
 * another block's values (Sec. 2's filter applied block-locally, the halo
 * values coming from the delayed levels), so one workgroup per block and
 * variable runs the x, y and z passes on an LDS copy of the block and writes
 * the filtered boundary layers to the ring, in place of three per-axis
 * launches and the ring fill.  Same arithmetic, so the same bits either way.
 * Applied to 3-D contexts whose blocks are all cubes of side 8, 16 or 32
 * (at most 16 in double precision); other contexts, synchronous steps and
 * atns_filter_state() take the per-axis passes.  Errors: ATNS_EINVAL for a
 * null context. */
atns_status atns_set_filter_fusion(atns_ctx* ctx, int32_t on);

/* Advance nsteps free-running asynchronous steps: the synchronization-
 * avoiding algorithm (Alg. 3) with delays that arise from the run itself
 * instead of a schedule.  One persistent workgroup per block advances its
 * block without grid-wide barriers; after each step it publishes the ring
 * level it has written.  At step n the delay from neighbour q is
 * k = max(0, n - m), m the newest level q has published, and the block
 * waits while k > L - 1 (with the guard of Alg. 3 this keeps k <= L - 1).
 * Euler or 3-D Navier-Stokes contexts in mode ATNS_AT or ATNS_AS with
 * ATNS_RK4 or ATNS_LSERK2;
 * the learned halo must be off; the history must hold C + L - 1 levels
 * (ESTATE otherwise).  The ring keeps C + 2L - 1 levels so that a neighbour
 * running L - 1 steps ahead never overwrites a level still needed.
 * dev_log: caller-owned device int8 array [nsteps][nblocks][ATNS_NSLOTS]
 * that receives the realized delays (-1 for slots the physics does not use);
 * replaying them through atns_set_delays and atns_rk_step reproduces the
 * run.  spin_limit: polls (each a short sleep) a workgroup waits for a
 * neighbour before the run is abandoned; every workgroup then leaves, the
 * call returns ATNS_ESTATE and the state must be set again.  EINVAL when
 * the blocks outnumber the workgroups that fit on the device at once (all
 * must be resident).  Synchronizes with the context stream. */
atns_status atns_step_async(atns_ctx* ctx, int32_t nsteps, int64_t spin_limit, int8_t* dev_log);

/* FP64 diagnostics of the current state (Sec. 5.2), into host_out[7]:
 * the five conserved totals sum U_v dV, the volume-averaged kinetic energy
 * (1/2V) int rho|u|^2 dV and enstrophy (1/2V) int rho|w|^2 dV, vorticity
 * by CD4 on the synchronous global field.  Synchronizes.  Returns
 * ATNS_ENONFINITE (with the values still written) if any value is not
 * finite, and ATNS_EINVAL for grids with 5 nx ny nz >= 2^31 points (the
 * kernel's 32-bit offsets; 512^3 fits). */
atns_status atns_reduce(atns_ctx* ctx, double* host_out);

/* atns_reduce for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops): the same FP64 diagnostics of a
 * field the caller owns, with no context, no allocation and no host
 * synchronization.  dev_U: device field in the field layout, float
 * (ATNS_F32) or double (ATNS_F64), ndim 2 or 3, n[3] points (nz == 1 in 2-D,
 * at least 5 per active axis), len[3] periodic box lengths.  dev_out: device
 * array of 7 doubles, written in the order of atns_reduce (no finiteness
 * check).  Enqueued on `stream` (hipStream_t or NULL).  The kernels' 1024
 * workgroup partial sums (57 KiB of doubles) live in a fixed device array that
 * every GPU the library runs on holds until the process ends; calls that
 * overlap on one GPU share it and race, so order them on one stream.  Results
 * equal atns_reduce's on the same field bit for bit.  Errors: EINVAL for null
 * pointers, bad precision or ndim, or grids with 5 nx ny nz >= 2^31 (the
 * kernels' 32-bit offsets); EHIP for a failed launch. */
atns_status atns_reduce_noalloc(const void* dev_U, int32_t precision, int32_t ndim, const int32_t* n,
                                const double* len, double* dev_out, void* stream);

/* Number of blocks, and the ring depth D (levels kept), of a context. */
atns_status atns_get_layout(const atns_ctx* ctx, int32_t* nblocks, int32_t* ring_depth);

/* Graph-captured steps (on by default).  Each asynchronous step (step >= C)
 * is one hipGraph launch: delay draw, halo assembly (and the learned-halo
 * correction when enabled), the s stage kernels and an increment of a device
 * step counter the kernels read, so one captured graph serves every step.
 * Synchronous steps, steps with injected delays and profiled steps run
 * eagerly.  The graph is re-captured after changes of dt, tile shape or the
 * learned-halo settings.  on = 0 runs every step eagerly.  Results are the
 * same bits either way. */
atns_status atns_set_graphs(atns_ctx* ctx, int32_t on);

/* Per-kernel timing of the fused stage kernels.  While enabled (on != 0),
 * the stage-kernel launches of each atns_rk_step step (and each atns_rhs
 * launch) are bracketed by a pair of HIP events recorded on the context
 * stream, one before the step's first stage launch and one after its last,
 * with no other work in between; the time includes the short gaps between
 * back-to-back launches.  atns_profile_read synchronizes, returns the number
 * of timed launches and their summed duration in ms, and clears the record.
 * Disabling also clears it. */
atns_status atns_profile_enable(atns_ctx* ctx, int32_t on);
atns_status atns_profile_read(atns_ctx* ctx, int64_t* launches, double* total_ms);

/* Tile shape of the stage kernels: a workgroup walks a TX x TY column of one
 * block through TZ planes.  Supported (TX, TY): Euler (16,16) (32,8) (16,8)
 * (64,8) (32,16); Navier-Stokes (16,16) (32,8) (16,8), and (32,16) in single
 * precision.  Tiles never straddle
 * blocks; ragged edges are handled.  EINVAL for other shapes or tz < 1. */
atns_status atns_set_tiles(atns_ctx* ctx, int32_t tx, int32_t ty, int32_t tz);
atns_status atns_get_tiles(const atns_ctx* ctx, int32_t* tx, int32_t* ty, int32_t* tz);

/* Autotuner of the tile shape.  Times every supported (TX, TY) with column
 * lengths TZ in {4, 8, 16, 32} (Navier-Stokes: 8, 16, 32) on the current
 * state -- reps times one step's mix of stage kernels (first, middle and
 * last RK stage, with the ring write), HIP events on the context stream,
 * writing only buffers that are dead at a step boundary (stage registers,
 * accumulator, the ring slot of level n + 1), so the state and the next
 * step are untouched -- and
 * keeps the fastest.  cache_path (or NULL) names a text file of
 * "key tx ty tz" lines; a configuration found there is applied without
 * timing, a newly tuned one is appended.  best_txyz (or NULL) receives the
 * chosen shape.  Synchronizes; ESTATE before a state is set. */
atns_status atns_autotune(atns_ctx* ctx, int32_t reps, const char* cache_path, int32_t* best_txyz);

/* ---- learned halo correction (an addition to the paper's method) --------
 * A 64-64-64-16 MLP (ReLU, BF16 operands on the matrix cores, FP32
 * accumulation) predicts, for each face halo point, the error of the AT
 * buffer extrapolation (Eq. 15) from the delayed levels the extrapolation
 * reads: features (U^{n-k-l}_v(p) - U^{n-k}_v(x)) / s_v for the 4 newest
 * levels l, the 5 variables v and the point x with its two neighbours p
 * along the face normal (60 values), then k/(L-1), then 3 zeros.  The
 * correction delta_v = r_v out_v is added to every stage halo value of the
 * point, unless |out_1..5|_2 > tau, when the AT value is kept (fallback).
 * Parameters: float[9360] = W1[64][64] b1[64] W2[64][64] b2[64] W3[16][64]
 * b3[16], row-major [out][in].  Training samples come from the context's
 * ring (an AT run, or an SA run created with L > 1, which keeps a history):
 * a random face halo point and delay k, target (U^n - Uhat_AT^(0)) / r_v.
 * X arrays are float[n][64], Y arrays float[n][8] (first 5 used). */
atns_status atns_mlp_set_params(atns_ctx* ctx, const float* host_params);
atns_status atns_mlp_get_params(atns_ctx* ctx, float* host_params);
/* Per-variable feature scales s_v and target scales r_v (positive). */
atns_status atns_mlp_set_scales(atns_ctx* ctx, const float* feat_scale5, const float* targ_scale5);
/* Outputs float[n][16] of the network for inputs dev_X (device). */
atns_status atns_mlp_forward(atns_ctx* ctx, const float* dev_X, int32_t n, float* dev_out);
/* Gradient (float[9360], device) and loss (mean over samples and the 5 used
 * outputs of the squared error) for one batch; deterministic. */
atns_status atns_mlp_grad(atns_ctx* ctx, const float* dev_X, const float* dev_Y, int32_t n, float* dev_grad,
                          double* host_loss);
/* n training samples (features, targets) from the current history with a
 * SplitMix64 stream seeded by `seed`.  ESTATE without a long enough ring. */
atns_status atns_mlp_sample(atns_ctx* ctx, int32_t n, uint64_t seed, float* dev_X, float* dev_Y);
/* `iters` Adam steps (beta 0.9/0.999, eps 1e-8) on fresh batches of `batch`
 * (>= 64) samples from the current history; host_losses (or NULL) receives
 * each batch's loss before its update.  Synchronizes. */
atns_status atns_mlp_train(atns_ctx* ctx, int32_t iters, int32_t batch, double lr, uint64_t seed,
                           double* host_losses);
/* Use the correction in every asynchronous step (mode ATNS_AT only). */
atns_status atns_mlp_enable(atns_ctx* ctx, int32_t on, double tau);
/* Corrected and fallback face-halo points since the last call (resets). */
atns_status atns_mlp_stats(atns_ctx* ctx, int64_t* applied, int64_t* fallback);

/* HBM probe: enqueue a plain streaming copy of `bytes` (a positive multiple
 * of 16) from dev_src to dev_dst on `stream` (hipStream_t or NULL).  Times
 * the achievable bandwidth and calibrates byte counters.  Buffers are the
 * caller's; nothing is allocated.  Asynchronous. */
atns_status atns_hbm_probe(const void* dev_src, void* dev_dst, int64_t bytes, void* stream);

/* ---- host-only helpers (no device needed) -------------------------------
 * The FP64 per-stage halo weight table the kernels use: out[e][k][l] for
 * stages e < s (s = 4 for RK4, 5 for LSERK4, 2 for LSERK2), delays k < L
 * and levels l < C (C = 5, or 3 for LSERK2).  AT: the buffer extrapolation
 * (stage 0, Eqs. 14-15) and the RK-consistent buffer updates (Eqs. 8-13,
 * App. C) in closed form; AS: 1 at l = 0.  out must hold s*L*C doubles. */
atns_status atns_host_weights(int32_t rk, int32_t mode, int32_t L, double* out);

/* The delays step n would draw (after the guard), without a device, into
 * out[nblocks][ATNS_NSLOTS]; *synchronous = 1 (and zeros) when n < C, C the
 * level count of scheme rk (5, or 3 for ATNS_LSERK2).  CAA: k = (n - C) mod
 * L everywhere.  SAA: SplitMix64 draw number (n*nblocks + b)*ATNS_NSLOTS + v
 * of stream `seed`, modulo L.  Then the guard of Alg. 3: k = 0 where
 * k > n - C + 1. */
atns_status atns_host_delays(int32_t algo, int32_t rk, int64_t n, int32_t nblocks, int32_t L,
                             uint64_t seed, int8_t* out, int32_t* synchronous);

/* ---- batches --------------------------------------------------------------
 * Many independent instances (members) -- different grids, block splits,
 * physics and delay bounds -- advanced together.  Members are ordinary
 * contexts (reach them with atns_batch_member to set state and dt, read
 * state and diagnostics) that must be three-dimensional, use classical RK4
 * and one precision, and
 * are stepped in lockstep by atns_batch_step.  After the first C
 * (synchronous) steps, which run member by member, every step is one
 * hipGraph launch in which a persistent, grid-stride stage kernel per physics
 * walks the combined tile list of all members of that physics; the Euler and
 * Navier-Stokes members form two independent branches of the graph.  Each
 * physics uses one tile shape for all its members (atns_batch_set_tiles, or
 * atns_batch_autotune, which times every shape with the batch kernels
 * themselves over all members of each physics -- one step's stage-kernel mix
 * writing only stage registers, as for atns_autotune, so no state changes --
 * then times the three fastest shapes of each physics in pairs, the two
 * physics running concurrently as in a batch step, and applies the fastest
 * pair; best receives int[6] = Euler (tx, ty, tz), Navier-Stokes
 * (tx, ty, tz)).  The persistent grid of each physics is as many workgroups
 * as the device holds at once for that kernel and shape.
 * Member results are bit-identical to stepping each member alone.
 * Ownership: the batch owns its member contexts; never pass a member to
 * atns_destroy (atns_batch_destroy releases them).  Member calls that change
 * dt, tiles or learned-halo settings are picked up by the next batch step
 * (the batch graph is re-captured).  atns_batch_step enqueues on internal
 * streams ordered after earlier work on the stream given at creation, and
 * later work on that stream is ordered after it.  Errors: ATNS_EINVAL for
 * bad arguments or members that are not 3-D classical RK4 of one precision,
 * ATNS_ESTATE if members are at different steps or lack state or dt
 * (atns_batch_autotune: lack state), ATNS_EHIP
 * for HIP failures; atns_batch_last_error(NULL) explains a failed create. */
typedef struct atns_batch atns_batch;
atns_status atns_batch_create(const atns_config* cfgs, int32_t n, void* stream, atns_batch** out);
atns_status atns_batch_destroy(atns_batch* batch);
const char* atns_batch_last_error(const atns_batch* batch);
atns_status atns_batch_member(atns_batch* batch, int32_t i, atns_ctx** ctx);
atns_status atns_batch_set_tiles(atns_batch* batch, int32_t physics, int32_t tx, int32_t ty, int32_t tz);
atns_status atns_batch_autotune(atns_batch* batch, int32_t reps, int32_t* best);
atns_status atns_batch_step(atns_batch* batch, int32_t nsteps);

#ifdef __cplusplus
}
#endif
#endif /* ATNS_H */
