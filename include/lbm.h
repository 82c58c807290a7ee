/*
 * lbm.h -- C ABI of the MI355X (gfx950) thermal lattice Boltzmann library.
 *
 * The library advances the discrete populations of a high-order thermal
 * lattice Boltzmann model with a body force, following Li & Shan, "Body-force
 * modelling in thermal compressible flows with lattice Boltzmann method"
 * (arXiv:2302.04741):
 *   - velocity sets: D2Q37 (degree-9 Gauss-Hermite rule, Sec. 3) and D3Q39
 *     (degree-7 rule, same construction as Sec. 2);
 *   - equilibrium: the Hermite expansion of the Maxwellian to order N,
 *     eq. (fN) with the coefficients a_0^(n) of Sec. 2 (N = 4 on D2Q37,
 *     N = 3 on D3Q39 by default);
 *   - body force: the Hermite expansion eq. (F), up to the third moment
 *     including the non-equilibrium stress, eq. (fi);
 *   - time step: eq. (lbm) with second-order time treatment: equilibrium and
 *     force evaluated at the mid-point values rho, u + g/2, theta and the
 *     mid-point stress sigma-bar of Sec. 2; BGK relaxation time tau-hat.
 * One step is one fused GPU kernel: pull streaming, moments, equilibrium,
 * stress, force, relaxation and the write of the new populations.
 *
 * Units: velocities in units of sqrt(theta_0) (theta_0 = 1), time in steps,
 * lengths in lattice nodes; g is the velocity increment per step.  Every grid
 * is periodic in every axis.
 *
 * Memory: the caller owns all device memory.  The library never allocates or
 * frees device memory: the state lives in a caller-provided workspace of
 * lbm_workspace_bytes() bytes.  Every call that takes device pointers runs
 * asynchronously on the handle's HIP stream, except lbm_totals, which
 * synchronises that stream to return host values.
 *
 * Errors: calls return an lbm_status; argument errors are detected
 * synchronously, before any GPU work is queued, and leave the handle
 * unchanged.  lbm_last_error() returns a thread-local message for the last
 * failure on the calling thread.  A handle is not thread-safe; distinct
 * handles are independent.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define LBM_API __attribute__((visibility("default")))
#else
#define LBM_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbm_sim lbm_sim; /* opaque host handle */

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,       /* invalid argument (null pointer, bad size, bad value) */
    LBM_EUNSUPPORTED = -2, /* valid request the library does not implement */
    LBM_EDEVICE = -3,      /* a HIP call failed; see lbm_last_error() */
    LBM_ENOSPACE = -4,     /* workspace too small */
    LBM_ENONFINITE = -5    /* a global total is NaN or infinite (diverged run) */
} lbm_status;

typedef enum { LBM_D2Q37 = 0, LBM_D3Q39 = 1 } lbm_lattice;

/* Population storage.  Arithmetic runs in FP64 for LBM_F64 and FP32 for
 * LBM_F32 and LBM_F16DEV.  Every storage type holds h_i = f~_i - w_i rho0
 * (see lbm_params.rho0); LBM_F16DEV stores h_i scaled by 2^k_i, k_i =
 * round(-log2 w_i), as IEEE half, so that deviations stay normal numbers.
 * The step stores LBM_F16DEV values with stochastic rounding (up or down with
 * probabilities that make the rounding error zero-mean; lbm_round_f16_stochastic
 * applies the same rounding to plain arrays), its random bits drawn from a
 * hash of (cell, step number) walked once per population: deterministic, and
 * independent of launch shape, batching and the other members; the initial
 * state rounds to nearest. */
typedef enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F16DEV = 2 } lbm_storage;

/* Truncation of the force expansion eq. (F).  The paper's N = 0, 1, 2 are
 * orders 1, 2, 3 here; "N = 2 without sigma" is LBM_FORCE_N2_NOSIGMA.
 * LBM_FORCE_N1_GUO keeps the first two moments only (Guo's scheme, i.e. the
 * force without a3_F). */
typedef enum {
    LBM_FORCE_N0 = 1,
    LBM_FORCE_N1_GUO = 2,
    LBM_FORCE_N2_NOSIGMA = 3,
    LBM_FORCE_N2 = 4
} lbm_force_order;

typedef enum { LBM_G_UNIFORM = 0, LBM_G_AXIS_PROFILE = 1, LBM_G_FIELD = 2 } lbm_force_kind;

/* lbm_params.flags */
#define LBM_FLAG_FORCE_FIELD 1u /* reserve workspace for an LBM_G_FIELD force */
#define LBM_FLAG_WALLS 2u       /* reserve workspace for plates (lbm_set_walls) */

typedef struct {
    uint32_t struct_size; /* = sizeof(lbm_params); ABI versioning */
    int32_t lattice;      /* lbm_lattice */
    int32_t storage;      /* lbm_storage */
    int32_t eq_order;     /* 0 = highest the rule supports (4 D2Q37, 3 D3Q39); else 2..that */
    int32_t force_order;  /* lbm_force_order; LBM_FORCE_N2 is the full scheme */
    uint32_t flags;       /* LBM_FLAG_* */
    int64_t nx, ny, nz;   /* grid extents, >= 1; nz == 1 for D2Q37; ny, nz <= 65535 */
    double tau_hat;       /* relaxation time of eq. (lbm), tau-hat = tau + 1/2; > 0.5 */
    double rho0;          /* reference density, >= 0: populations are stored and
                             advanced as deviations h_i = f~_i - w_i rho0.  rho0 = 1
                             keeps every stored value and every rounding at the size
                             of the deviations; rho0 = 0 stores f~ itself (the
                             literal form of eq. (lbm)). */
} lbm_params;

/* Bytes of device workspace a handle needs for these parameters (256-byte
 * aligned sub-buffers included): two arrays of the Q populations f~_i of
 * eq. (lbm), in planes whose rows are padded to a multiple of 64 values, the
 * force table, the reduction scratch of lbm_totals and a step counter (with LBM_FLAG_WALLS
 * also the plates' row sums and emission tables).  Returns 0 if the
 * parameters are invalid. */
LBM_API size_t lbm_workspace_bytes(const lbm_params *p);

/* Create a handle and initialise the populations from FP64 device fields.
 *   workspace : device memory of >= lbm_workspace_bytes(p) bytes, 256-byte
 *               aligned, owned by the caller, not freed by the library; it
 *               must stay valid until lbm_destroy.
 *   hip_stream: the hipStream_t every call of this handle runs on (NULL = the
 *               null stream).
 *   rho, theta: N = nx*ny*nz doubles; u: D*N doubles (component-major, u[a*N +
 *               cell]); cell = (z*ny + y)*nx + x.  Read by an init kernel queued
 *               on hip_stream: the caller may reuse them once that stream
 *               has passed this call.
 * The initial stored state is f~ = f0(rho, u, theta) - F/2 (the auxiliary
 * variable of eq. (lbm) at n = 0, with f0 of eq. (fN) and F of eq. (fi) at
 * sigma = 0) with the current force (zero until lbm_set_force), so
 * lbm_moments reports exactly the inputs at step 0.  Returns LBM_EINVAL / LBM_EUNSUPPORTED / LBM_ENOSPACE without
 * queuing work, LBM_EDEVICE if the launch fails. */
LBM_API lbm_status lbm_create(const lbm_params *p, void *workspace, size_t workspace_bytes,
                      void *hip_stream, const double *rho, const double *u,
                      const double *theta, lbm_sim **out);

/* Set the body acceleration g (Sec. 2, eq. (BGK): the acceleration of the body
 * force).  kind:
 *   LBM_G_UNIFORM      g: D host doubles; axis and len ignored.
 *   LBM_G_AXIS_PROFILE g: D*len device doubles, g[a*len + k] = g_a at
 *                      coordinate k along `axis` (0 = x, 1 = y, 2 = z);
 *                      len must equal that grid extent.
 *   LBM_G_FIELD        g: D*N device doubles, g[a*N + cell]; needs
 *                      LBM_FLAG_FORCE_FIELD at creation.
 * Device data are copied (and converted to the arithmetic precision) into the
 * workspace on the handle's stream; the caller may reuse them afterwards.
 * Before the first step the stored state is rebuilt from its moments so that
 * f~ = f0 - F/2 holds with the new g (the moments reported at step 0 stay the
 * initial ones); after that, g applies from the next step on. */
LBM_API lbm_status lbm_set_force(lbm_sim *s, int32_t kind, const double *g, int32_t axis, int64_t len);

/* Advance nsteps (>= 0) time steps of eq. (lbm); asynchronous.  If a launch
 * fails (LBM_EDEVICE), the steps enqueued before it still run and are counted
 * in lbm_step_count. */
LBM_API lbm_status lbm_step(lbm_sim *s, int64_t nsteps);

/* Physical moments at the current step, eq. (rut1) with the mid-point shift:
 * rho, u = u~ + g/2 and theta (the mid-point values of Sec. 2).  Device FP64
 * outputs: rho[N], u[D*N] (component-major), theta[N]; any may be NULL. */
LBM_API lbm_status lbm_moments(lbm_sim *s, double *rho, double *u, double *theta);

/* Destroy the handle (NULL is a no-op; housekeeping, no passage of the paper).
 * Does not free the workspace and does not wait for queued work; the
 * workspace may be reused once the stream has drained. */
LBM_API void lbm_destroy(lbm_sim *s);

/* Thread-local message of the last failed call ("" if none; housekeeping). */
LBM_API const char *lbm_last_error(void);

/* ---- diagnostics, checkpointing and tables (not part of the step path) ---- */

/* Global sums over the grid of the stored populations (the moments of
 * eq. (rut1) summed over all cells: mass, momentum and twice the energy of f~),
 * reduced in FP64 in a fixed order (bitwise reproducible):
 * out[0] = sum f~, out[1..D] = sum f~ xi_a, out[D+1] = sum f~ |xi|^2 (host,
 * D+2 doubles).  Synchronises the handle's stream.  Returns LBM_ENONFINITE if
 * any sum is not finite. */
LBM_API lbm_status lbm_totals(lbm_sim *s, double *out);

/* The same sums as lbm_totals, written to device memory and not waited for:
 * out_dev receives D+2 doubles on the handle's stream (asynchronous, no
 * finiteness check), so that a caller can check many simulations without
 * stalling the device (a serving loop reads them back once their step work is
 * done).  LBM_EINVAL on a NULL handle or pointer. */
LBM_API lbm_status lbm_totals_device(lbm_sim *s, double *out_dev);

/* Heat flux q = 1/2 sum_i f_i |xi_i - u|^2 (xi_i - u) of the physical
 * distribution f = f0 + (1 - 1/(2 tau-hat)) (f~ - f0 + F/2) at the current
 * step (the quantity q_err of Sec. 2 refers to).  q: D*N device doubles. */
LBM_API lbm_status lbm_heat_flux(lbm_sim *s, double *q);

/* The rounding the step applies when it stores F16 deviations
 * (LBM_F16DEV): each of n FP32 values v[k] becomes a binary16 out[k] (bit
 * pattern) by stochastic rounding -- a value between neighbouring halves
 * a < v < b becomes b with probability (v - a)/(b - a), so the rounding error
 * has zero mean -- with seed[k] as its random bits.  In the normal half range
 * the result is: add seed[k] >> 19 to the FP32 bit pattern (sign and
 * magnitude) below the 13 bits binary16 drops, then drop them; below 2^-14 the
 * rounding is stochastic at the subnormal spacing 2^-24.  Values a half holds
 * exactly are returned unchanged.  v, seed and out are device arrays of n
 * elements (out may not overlap the inputs); the call is enqueued on
 * hip_stream (NULL: the null stream) and not waited for.  For callers that
 * encode F16 deviations themselves, and for tests of the rounding.
 * LBM_EINVAL if n < 0, or n > 0 with a NULL pointer; n = 0 does nothing. */
LBM_API lbm_status lbm_round_f16_stochastic(const float *v, const uint32_t *seed, uint16_t *out,
                                            int64_t n, void *hip_stream);

/* Access-pattern diagnostic: `repeats` passes of the memory traffic of the
 * step alone -- the streaming of eq. (lbm): every population read from its
 * pull source x - c_i and written back unchanged at the cell's own slot of
 * the idle population buffer, with the step's work split and launch shape but
 * none of its arithmetic.  The state, the step count and everything a later
 * call reads are unchanged (a step overwrites the idle buffer whole).  Timing
 * it beside lbm_step gives the ceiling of the step's access pattern on the
 * device.  Async on the handle's stream; LBM_EINVAL if repeats < 0. */
LBM_API lbm_status lbm_pattern_pass(lbm_sim *s, int64_t repeats);

/* Raw population state for checkpoint/restart (the stored f~_i of eq. (lbm),
 * as deviations): lbm_population_bytes bytes, dense SoA planes of h_i in the
 * storage type, value i*N + cell (the padding
 * of the internal rows is dropped), post-collision "pull" layout.  get copies
 * out, set copies in (device buffers, async on the handle's stream).
 * Restoring a state together with lbm_set_step_count resumes bitwise (with
 * F16 storage the step number keys the stochastic rounding: set_step_count
 * also sets the device counter, asynchronously on the handle's stream). */
LBM_API size_t lbm_population_bytes(const lbm_sim *s);
LBM_API lbm_status lbm_get_populations(lbm_sim *s, void *dst);
LBM_API lbm_status lbm_set_populations(lbm_sim *s, const void *src);
LBM_API int64_t lbm_step_count(const lbm_sim *s);
LBM_API lbm_status lbm_set_step_count(lbm_sim *s, int64_t n);

/* Change the stream of a handle (work already queued stays where it is;
 * housekeeping, no passage of the paper). */
LBM_API lbm_status lbm_set_stream(lbm_sim *s, void *hip_stream);

/* Kernel launch shape of the step of eq. (lbm) (an implementation choice, not
 * the paper's): threads per block (64, 128, 256, 512 or
 * 1024; FP64 storage uses at most 256), i.e. wavefronts per block, each
 * wavefront updating 64 consecutive cells of one row.  0 restores the default
 * (256; 128 for FP64 storage; 1024 for D3Q39 FP32 grids of at least 2^17
 * wavefronts).  Results do not depend on it. */
LBM_API lbm_status lbm_set_block(lbm_sim *s, int32_t threads);

/* Relaxation time per cell (Sec. 3 of the paper: tau = mu/(rho theta) keeps the
 * dynamic viscosity mu and the heat conductivity constant).  mu > 0: every
 * step, the stress and the heat flux use tau^ = mu/(rho theta) + 1/2 with the
 * cell's own mid-point rho and theta (tau^ = tau + 1/2 as in eq. (lbm)); the
 * tau_hat of the parameters is ignored until mu is set back to 0.  mu is in
 * the units of tau_hat * theta (time steps times reference temperature).
 * Takes effect at the next step; batches and graphs that hold the handle must
 * be rebuilt (they refuse to run stale).  LBM_EINVAL if mu < 0 or not finite. */
LBM_API lbm_status lbm_set_viscosity(lbm_sim *s, double mu);

/* Plates normal to y, for the channel flow of Sec. 3 (the paper does not
 * publish its wall condition; this one is the library's own).  enable != 0
 * puts plates at y = -1/2 and y = ny - 1/2 (x and z stay periodic) with
 * temperatures theta_b, theta_t (> 0) and tangential velocities u_b, u_t along
 * x.  Diffuse reflection with exact mass conservation: every population that
 * would stream into a plate is absorbed, its mass credited to the (x, z)
 * column of the node it leaves; the plate emits f0_i(1, (u_w, 0, 0), theta_w)
 * times a per-column density into every slot whose streaming source lies
 * behind it, the density fixed so that each column re-emits exactly what it
 * absorbed.  Needs LBM_FLAG_WALLS at creation and step count 0; the state is
 * rebuilt from the moments the handle reports (f~ = f0 - F/2 at every node,
 * then the populations that would come from behind a plate replaced by its
 * emission balancing the initial outgoing populations).  A step with plates is
 * still one launch: the step that writes a state also writes, per row next to
 * a plate, the sums the next step's emission needs.  enable = 0 removes the
 * plates.  Handles with plates may join a batch (their plates included).
 * LBM_EINVAL on bad values, a missing flag or a stepped handle. */
LBM_API lbm_status lbm_set_walls(lbm_sim *s, int32_t enable, double theta_b, double theta_t,
                                 double u_b, double u_t);

/* ---- batching: several simulations per launch, and captured step loops ---- */

typedef struct lbm_batch lbm_batch; /* opaque host handle */
typedef struct lbm_graph lbm_graph; /* opaque host handle */

/* Device workspace of a batch of up to max_sims simulations (execution only,
 * no passage of the paper; its tile table:
 * 8 * (max_sims + 1) bytes of tile offsets, rounded up to 256, then one
 * descriptor per member). */
LBM_API size_t lbm_batch_workspace_bytes(int32_t max_sims);

/* A batch advances its member simulations together, each by eq. (lbm) exactly
 * as lbm_step does (an execution choice; the paper treats one grid): every step
 * is ONE launch
 * of a multi-grid kernel over a list of tiles spanning all members (one tile =
 * 64 consecutive cells of one grid row of one member, updated by one
 * wavefront).  By default every tile gets its own wavefront and the hardware
 * balances uneven members; with a block count set, a persistent grid walks the
 * list with a fixed stride.
 * Members must share lattice, storage, eq_order and force_order; grid sizes,
 * tau_hat, mu, rho0, forces and plates may differ.  The per-cell arithmetic is
 * that of lbm_step, so a member's result does not depend on the other members
 * or on the launch shape.  Runs on hip_stream. */
LBM_API lbm_status lbm_batch_create(int32_t max_sims, void *workspace, size_t workspace_bytes,
                                    void *hip_stream, lbm_batch **out);

/* Set the members (1..max_sims handles, no duplicates) and write the tile
 * table on the batch's stream (small copy kernels; the call does not wait for
 * the device).  Call again after a member was stepped or had
 * its force changed outside the batch (lbm_batch_step refuses stale tables).
 * Destroying a member leaves the batch unusable until the next lbm_batch_set. */
LBM_API lbm_status lbm_batch_set(lbm_batch *b, lbm_sim *const *sims, int32_t count);

/* Advance every member by nsteps (>= 0) steps of eq. (lbm), one launch per
 * step, on the batch's stream.  The library does not order that stream with the members'
 * own streams: work queued on a member's stream must be complete (or ordered
 * with events) before, and later work on it must wait for the batch's stream
 * (the Python binding does both).  If a launch fails (LBM_EDEVICE), the steps
 * enqueued before it still run and are counted in every member's state. */
LBM_API lbm_status lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Launch shape of the multi-grid kernel (an implementation choice).  threads: threads per block, 64, 128
 * or 256 (0 = 128), i.e. 1, 2 or 4 tiles per block; blocks: 0 = enough blocks
 * for one wavefront per tile (default), > 0 = a persistent grid of that many
 * blocks (at most 2^31 - 1).  Results do not depend on the shape.  Graphs
 * captured before must be captured again. */
LBM_API lbm_status lbm_batch_set_launch(lbm_batch *b, int32_t threads, int64_t blocks);

/* Housekeeping; NULL-safe; does not free the workspace and does not wait for
 * queued steps (the caller keeps the workspace until the stream has run them). */
LBM_API void lbm_batch_destroy(lbm_batch *b);

/* Largest member count of lbm_batch_step_noalloc. */
#define LBM_NOALLOC_MAX_SIMS 256

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): advance `count`
 * simulations by nsteps (>= 0) steps of eq. (lbm) in the multi-grid kernel of
 * lbm_batch_step, with no batch handle and no batch workspace.  The tile table
 * (the scratch of the multi-grid kernel: tile offsets and one descriptor per
 * member) lives in a fixed device array of the library, sized for
 * LBM_NOALLOC_MAX_SIMS members (about 51 KB; each device the library runs on
 * holds one until the process ends).  Every call rewrites that table on
 * hip_stream with small copy kernels (the descriptors travel as kernel
 * arguments, so no host buffer must outlive the call), then launches one
 * multi-grid step per step.
 *   sims: 1..LBM_NOALLOC_MAX_SIMS distinct handles sharing lattice, storage,
 *         eq_order and force_order (grids, tau_hat, mu, forces and plates may
 *         differ); count above the maximum is LBM_EINVAL.  Launch shape: that
 *         of a default batch (128 threads, one wavefront per 64-cell tile), so
 *         every member's result is bitwise the one lbm_batch_step gives.
 *   hip_stream: the stream of every launch (NULL = the null stream); the
 *         current device must be the members' device.  As with lbm_batch_step,
 *         work on the members' own streams must be ordered with it by the caller.
 * No call allocates or frees memory on the device or the host.  The array is
 * shared by every call on a device and keeps the last call's table: calls that
 * overlap on one device (different streams, or threads) race and must be
 * serialised by the caller.  The first call on a device resolves the array's
 * address (hipGetSymbolAddress); make it once before any graph capture.
 * Errors: as lbm_batch_step; argument errors leave every member unchanged. */
LBM_API lbm_status lbm_batch_step_noalloc(lbm_sim *const *sims, int32_t count, int64_t nsteps,
                                          void *hip_stream);

/* Capture nsteps (even, > 0) steps of eq. (lbm) of one simulation (s) or one
 * batch (b) --
 * exactly one of them non-NULL -- into a HIP graph on its stream, which must
 * not be the null stream.  Capturing executes nothing and leaves the state
 * unchanged.  The graph holds the buffers of the handle: it stays valid while
 * the handle lives and is not re-initialised (lbm_set_force before the first
 * step rebuilds in place, so it is fine; a new lbm_batch_set is not). */
LBM_API lbm_status lbm_graph_create(lbm_sim *s, lbm_batch *b, int64_t nsteps, lbm_graph **out);

/* Replay the captured steps of eq. (lbm) `repeats` times (asynchronous on the
 * stream).  If a replay fails to launch (LBM_EDEVICE), the replays enqueued
 * before it still run and are counted. */
LBM_API lbm_status lbm_graph_launch(lbm_graph *g, int64_t repeats);

/* Housekeeping; NULL-safe. */
LBM_API void lbm_graph_destroy(lbm_graph *g);

/* The velocity set compiled into the library (host call, no GPU needed): the
 * Gauss-Hermite rule of Sec. 2 (D2Q37 of Sec. 3, r ~ 1.19698; D3Q39 built the
 * same way).  c: Q*3 ints, w: Q doubles, r: the scale with xi_i = r c_i.  Returns Q, or a
 * negative lbm_status. */
LBM_API int32_t lbm_lattice_table(int32_t lattice, int32_t *c, double *w, double *r);

/* Library version string (housekeeping). */
LBM_API const char *lbm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
