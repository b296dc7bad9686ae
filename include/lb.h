/*
 * lb.h -- C ABI of the MI355X D3Q19 lattice Boltzmann library.
 *
 * The library advances a D3Q19 BGK lattice with the fused collide-and-stream
 * update of the paper (arXiv 2409.16781): Eq. 1 (lattice Boltzmann equation),
 * Eq. 2-3 (second-order equilibrium), Section 3.1 (fused kernel with a
 * scattered read from the pre-collision array, a write into the
 * post-collision array and a swap; one unit-stride vector per population),
 * Section 3.1.1 (storage precision, "Mixed1": half-precision storage with
 * single-precision arithmetic).  On top of the paper's two-dimensional method
 * it provides the three-dimensional D3Q19 velocity set, halfway bounce-back
 * at solid sites (the no-slip walls of Section 3.3), periodic faces, and a
 * uniform body force in Guo's form as the source term S_i of Eq. 1.
 *
 * Conventions shared by every call:
 *  - Lattice sites are indexed s = x + nx * (y + ny * z), x fastest.
 *  - Population order (also the layout of lb_get_f / lb_set_f):
 *      0 (0,0,0); 1 (+1,0,0); 2 (-1,0,0); 3 (0,+1,0); 4 (0,-1,0); 5 (0,0,+1);
 *      6 (0,0,-1); 7 (+1,+1,0); 8 (+1,-1,0); 9 (-1,+1,0); 10 (-1,-1,0);
 *      11 (+1,0,+1); 12 (+1,0,-1); 13 (-1,0,+1); 14 (-1,0,-1); 15 (0,+1,+1);
 *      16 (0,+1,-1); 17 (0,-1,+1); 18 (0,-1,-1).
 *    Weights: 1/3 (rest), 1/18 (axis), 1/36 (diagonal).
 *  - The stored state is the post-collision population array.  It is kept
 *    shifted by the lattice weights, g_i = f_i - w_i, in the storage codec
 *    chosen at creation (FP32, FP16 / BF16 rounded to nearest even, or the
 *    scaled 16-bit fixed point LB_S16); all arithmetic is FP32.
 *  - "Device" pointers are HIP device memory owned by the caller; the library
 *    never frees them.  Calls that take device pointers are enqueued on the
 *    lattice's stream and return before the work completes.
 *  - Every int-returning call returns LB_OK (0) or a negative status code and
 *    records a message readable with lb_last_error() on the calling thread.
 *    No C++ exception crosses this interface.
 *  - A handle may be used from one thread at a time; handles are independent.
 */
#ifndef LB_H
#define LB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lb_lattice lb_lattice;

/* Status codes. */
#define LB_OK 0
#define LB_EINVAL (-1)    /* an argument is out of range or inconsistent        */
#define LB_ENOMEM (-2)    /* device or host allocation failed                   */
#define LB_EHIP (-3)      /* a HIP runtime call failed (no device, launch error) */
#define LB_EUNSTABLE (-4) /* a conservation sum is NaN or infinite              */
#define LB_ESTATE (-5)    /* the handle is not a live lattice                   */

/* Storage codecs (Section 3.1.1: storage precision vs. arithmetic precision). */
#define LB_F32 0   /* FP32 storage of g = f - w, 4 bytes per population      */
#define LB_F16S 1  /* FP16 storage of g = f - w, round-to-nearest-even        */
#define LB_BF16S 2 /* BF16 storage of g = f - w, round-to-nearest-even        */
/*
 * LB_S16: scaled 16-bit fixed point of g = f - w (a custom 16-bit codec for
 * the storage-precision question of Section 3.1.1; arithmetic stays FP32).
 * Population i is stored as the int16 code q with g_i = q * 2^-e, with one
 * exponent e per weight class (rest, axis, diagonal) for the whole lattice.
 * lb_init_eq sizes each class from the initial state (|g_i| <= w_i 2^m with
 * 2^m at least twice the class's largest |g_i| / w_i).  Encoding rounds to
 * nearest even.  A step in which a code would leave [-32768, 32767] (or a
 * density is not finite) flags itself with the classes concerned; the steps
 * after it do nothing, and the next call that waits for the lattice
 * (lb_sync, lb_sums, lb_macros, lb_get_f, ...) widens those classes' ranges
 * by one bit, re-encodes the intact source array of the flagged step and
 * redoes the remaining steps, as often as needed (LB_EUNSTABLE past the
 * widest range).  Two-array storage only; not with force fields, the adjoint or the
 * outlet flux.  Raw words (lb_get_f) are the int16 codes; lb_get_scales gives
 * their exponents.
 */
#define LB_S16 3

/*
 * Flag OR-ed into the storage argument of lb_create_ex: keep ONE population
 * array instead of two (in-place update in the "AA" access pattern: steps
 * alternate between one that gathers from the neighbours and pushes back to
 * them and one that works at the site itself; every site reads and writes
 * the same 19 locations, so no second array is needed).  Half the memory,
 * the same bytes moved per step, results identical to two-array storage.
 * Needs rows that tile whole: nx = V * 2^k with nx / V <= 256 for V in
 * {4, 2, 1} (FP32) or {8, 4, 2} (16-bit codecs).  Not with force fields or
 * the adjoint.
 */
#define LB_INPLACE 0x100

/* Memory spaces for lb_get_f / lb_set_f. */
#define LB_HOST 0
#define LB_DEVICE 1

/*
 * Create a lattice of nx * ny * nz sites with relaxation time tau (omega =
 * 1/tau, kinematic viscosity (tau - 1/2)/3; Eq. 1).  tau must be > 0.5, or
 * +INFINITY, which gives omega = 0 (pure streaming).  flags is a HOST pointer
 * to nx*ny*nz bytes, 0 = fluid, 1 = solid (no-slip obstacle or wall; any other
 * value is rejected), copied by the call; NULL means all fluid.  Every face
 * is periodic.  The lattice starts at rest (g = 0) with zero force and FP32
 * storage, on the default HIP stream.  Device memory for two population
 * arrays and the flag masks is allocated here and owned by the lattice.
 * Returns NULL on failure (see lb_last_error()).
 */
lb_lattice *lb_create(int nx, int ny, int nz, double tau, const uint8_t *flags);

/*
 * As lb_create, with a storage codec (LB_F32, LB_F16S, LB_BF16S, LB_S16, optionally
 * OR-ed with LB_INPLACE) and a HIP stream (hipStream_t passed as void*) on
 * which all of the lattice's work is enqueued.  NULL is the default stream.  The stream is borrowed: the
 * lattice never destroys it, and it must outlive the lattice.
 */
lb_lattice *lb_create_ex(int nx, int ny, int nz, double tau, const uint8_t *flags, int storage,
                         void *hip_stream);

/* Release everything the lattice owns (waits for its stream first).  NULL is
 * a no-op.  A destroyed handle must not be used again. */
void lb_destroy(lb_lattice *lat);

/*
 * Uniform body-force density F (lattice units, per site per step), entering
 * as Guo's source term S_i = (1 - omega/2) w_i [3 (c_i - u) + 9 (c_i.u) c_i].F
 * with the velocity u = (sum_i c_i f_i + F/2) / rho (the paper's source term
 * S_i of Eq. 1, Section 2).  Applies to the steps enqueued after the call.
 */
int lb_set_force(lb_lattice *lat, double fx, double fy, double fz);

/*
 * Set the state to the equilibrium of Eq. 2-3 at every fluid site:
 * f_i = f_i^eq(rho, u), computed in FP64 and rounded once into the storage
 * codec.  rho: device array of N doubles (NULL: rho = 1); u: device array of
 * 3N doubles, component-major (N values of u_x, then u_y, then u_z; NULL:
 * u = 0).  Solid sites are set to rest.  Resets the step count to 0.
 */
int lb_init_eq(lb_lattice *lat, const double *rho, const double *u);

/*
 * Enqueue n >= 0 fused steps (Eq. 1, Section 3.1): for every fluid site x,
 *   f_i = S_i(x - c_i), or S_opp(i)(x) when x - c_i is solid (bounce-back),
 *   rho = sum f_i,  u = (sum c_i f_i + F/2)/rho,
 *   S'_i(x) = f_i - omega (f_i - f_i^eq) + S_i^F,
 * then swap the arrays.  Each step also records the FP64 totals of the new
 * state (see lb_sums).  A request of 64 or more steps runs as one captured
 * HIP graph of the whole request (at most 1024 steps per graph), kept and
 * replayed for the next request of the same length.
 */
int lb_step(lb_lattice *lat, int n);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same n
 * steps as lb_step, with the same results (state and totals bit for bit), but
 * the call allocates nothing.  The totals' scratch (the reduce's arrival
 * ticket and the per-workgroup FP64 partials) lives in a file-scope device
 * array of the library, 8 MiB + 64 KiB per device, held until the process
 * ends; each step is an ordinary kernel launch on the lattice stream (no
 * graph is built, so a caller may capture the call into its own).
 * Limit: 64 bytes per step workgroup plus 256 + 32 per 256 workgroups; a
 * 512^3 lattice at 4 sites per lane (131072 workgroups) fits, lattices that
 * need more are rejected with LB_EINVAL and the sizes in lb_last_error().  All calls on one device
 * share the one array, which keeps the last call's contents: calls that
 * overlap on one device (other streams, other threads) race and must not be
 * issued.  Call with the lattice's device current.
 */
int lb_step_noalloc(lb_lattice *lat, int n);

/*
 * As lb_step with n >= 1, and the last step also writes the density and
 * velocity it computes (the pre-collision moments of that step, u including
 * the half-force shift) into caller-owned device arrays rho (N floats) and u
 * (3N floats, component-major).  Solid sites get rho = 0, u = 0.  With
 * in-place storage (LB_INPLACE) the fields come from the state just written,
 * as lb_macros computes them (equal up to FP32 rounding).
 */
int lb_step_macros(lb_lattice *lat, int n, float *rho, float *u);

/*
 * Density and velocity of the current state (the macroscopic moments of
 * Section 2: density as the sum of the populations, momentum as their
 * velocity-weighted sum), into caller-owned device arrays rho (N floats) and
 * u (3N floats, component-major):
 *   rho = sum_i f_i,   u = (sum_i c_i f_i - F/2) / rho.
 * After a step these equal the pre-collision moments of that step (collision
 * keeps mass and the source adds exactly F to the momentum).  Solid sites get
 * rho = 0, u = 0.  Either pointer may be NULL to skip it.
 */
int lb_macros(lb_lattice *lat, float *rho, float *u);

/*
 * Copy the conservation totals of the last k steps into out[4*k] (host),
 * oldest first: {mass, momentum_x, momentum_y, momentum_z} summed over fluid
 * sites of each step's stored state (sum of f_i = w_i + g_i and of c_i g_i, as
 * stored): the moments of Section 2 summed over the lattice, which the
 * collision of Eq. 1 conserves (mass exactly, momentum up to the force F per
 * fluid site and step).  Every stored value is converted to FP64 and summed
 * in FP64 on the GPU in a fixed order (bitwise reproducible).  k must be <= min(steps taken since lb_init_eq, 4096).
 * Synchronises the stream.  Returns LB_EUNSTABLE when any copied value is
 * NaN or infinite (the values are still copied).
 */
int lb_sums(lb_lattice *lat, double *out, int k);

/*
 * Raw state in storage format: the post-collision array of the fused scheme
 * (Section 3.1: the array a step writes and the next step reads), e.g. for a
 * checkpoint and restart of a run.  19 planes of N elements (plane i =
 * population i, site order as above; the structure-of-arrays form of
 * Section 3.1), each element the codec's value of g_i = f_i - w_i
 * (float for LB_F32, IEEE binary16 for LB_F16S, bfloat16 for LB_BF16S).
 * bytes must equal 19 * N * (4 or 2).  where is LB_HOST or LB_DEVICE.
 * Host copies synchronise; device copies are enqueued.  lb_set_f leaves the
 * step count unchanged.  Values at solid sites are not part of the state: no
 * step reads them, and a step writes zero there (or leaves them unchanged).
 */
int lb_get_f(lb_lattice *lat, void *buf, size_t bytes, int where);
int lb_set_f(lb_lattice *lat, const void *buf, size_t bytes, int where);

/* Wait until all work enqueued on the lattice's stream has finished. */
int lb_sync(lb_lattice *lat);

/*
 * LB_S16 storage only: the 3 exponents of the stored codes, for the rest,
 * axis and diagonal populations (g_i = q_i 2^-e), after settling pending
 * steps.  lb_set_scales sets them without touching the stored words, for
 * restoring a checkpoint taken with lb_get_f and lb_get_scales (each in
 * [4, 60]).  Other codecs: LB_EINVAL.
 */
int lb_get_scales(lb_lattice *lat, int *exps);
int lb_set_scales(lb_lattice *lat, const int *exps);

/* Message of the last failing call on this thread ("" if none). */
const char *lb_last_error(void);

/* ---- queries and measurement helpers -------------------------------------- */

/* Number of steps taken since lb_init_eq (host count of enqueued steps). */
long long lb_steps_done(const lb_lattice *lat);

/*
 * Integer properties: key 0 = kernel variant of the step (0 = one site per
 * thread, 1 / 2 / 3 = vector rows with 16- / 8- / 4-byte accesses per lane
 * and population), 1 = sites per thread, 2 = 1 if the lattice has solid
 * sites, 3 = bytes per stored population, 4 = workgroups per step launch,
 * 5 = x-rows per storage block, 6 = number of fluid sites, 7 = bytes of one
 * population array, 8 = 1 for in-place (one-array) storage, 9 = storage
 * codec, 10 = range widenings of LB_S16 storage so far, 11 = tile order (0
 * linear, 1 a contiguous range of tiles per XCD, 2 linear with each block of
 * 64 tiles rotated by its index), 12 = 1 if the steps of a
 * lattice with solids pull with non-temporal loads (else cached loads).
 * Returns -1 for an unknown key or a bad handle.
 */
long long lb_query(const lb_lattice *lat, int key);

/*
 * Enqueue n steps between two HIP events recorded on the lattice's stream,
 * wait for them, and store the elapsed milliseconds in *ms.
 */
int lb_time_steps(lb_lattice *lat, int n, double *ms);

/*
 * Enqueue n steps one by one (no graph) with HIP events on the lattice's
 * stream around each step kernel alone (without the small kernel that adds
 * up the conservation totals), wait, and store the mean step-kernel duration
 * in milliseconds in *ms.  The state advances by n steps as with lb_step.
 */
int lb_time_step_kernel(lb_lattice *lat, int n, double *ms);

/*
 * Launch-shape tuner: time the step kernel with every vector width that
 * divides nx (16-, 8- and 4-byte accesses per lane) and the three tile
 * orders (lb_query key 11), with solids also both
 * cache policies of the pull loads (cached, or non-temporal), reps launches
 * each in two passes over the candidates, and keep the fastest for this
 * lattice (lb_query keys 0, 4, 11 and 12
 * report it).  Each
 * timing launch reads the current state and writes the other array, so the
 * state, the step count and the totals are unchanged.  Synchronises.  Not for
 * in-place storage (LB_EINVAL).
 */
int lb_tune(lb_lattice *lat, int reps);

/*
 * Bandwidth ceiling probe: a streaming copy (one 16-byte non-temporal load
 * and store per lane) of the current population array into the other one
 * (the same bytes a step reads and writes), run reps times between HIP
 * events on the lattice's stream.
 * Stores the mean milliseconds per copy in *ms.  Overwrites only the scratch
 * array, so the state is unchanged.
 */
int lb_copy_probe(lb_lattice *lat, int reps, double *ms);

/* ---- differentiation ----------------------------------------------------- */

/*
 * Per-site x-force: fx is a caller-owned DEVICE array of N floats (site
 * order), copied; from now on the force density of site s is
 * (F_x + fx[s], F_y, F_z) in the collision (Guo source and half-force
 * velocity shift, Eq. 1) and in lb_macros.  NULL removes the field.
 * FP32 storage only.  The copy is enqueued on the lattice's stream.
 */
int lb_set_force_field(lb_lattice *lat, const float *fx);

/*
 * Gradient of an objective of the final state with respect to the per-site
 * x-force, by the adjoint of the fused step (reverse mode: the transposed
 * collision Jacobian of BGK with Guo forcing and the transposed pull
 * streaming with bounce-back, one fused kernel per step).
 * The call advances the lattice by nsteps steps exactly as lb_step does
 * (state, step count and totals), keeping the state every `every` steps
 * (checkpoints) and the density and velocity of each step of the last
 * stretch, then sweeps backwards: each earlier stretch of `every` steps is
 * recomputed from its checkpoint, keeping its steps' density and velocity,
 * and differentiated.  seed: caller-owned DEVICE array of
 * 19 * N floats in the raw-state layout of lb_get_f holding dJ/dS_N, the
 * derivative of the objective with respect to the final stored state (zero
 * at solid sites).  grad: caller-owned DEVICE array of N floats, overwritten
 * with sum over the steps of dJ/dF_x(s) through the collisions; a term of J
 * that depends on the force directly is the caller's to add.  FP32 storage.
 * Device memory for ceil(nsteps / every) + 4 states and 16 * N *
 * min(every, nsteps) bytes is allocated by the first call that needs it and
 * kept by the lattice for later calls (lb_destroy frees it); the call
 * synchronises the stream.
 */
int lb_grad_force_x(lb_lattice *lat, int nsteps, int every, const float *seed, float *grad);

/*
 * The outlet mass flux of the current state: J = sum over the fluid sites of
 * the plane x = nx - 1 of rho u_x, with rho and u the moments of Section 2
 * (u including the half-force shift of Guo's source term, Eq. 1), i.e.
 * J = sum_i c_ix f_i - F_x / 2 per site with F_x the site's x-force.  Summed
 * in FP64 on the GPU in a fixed order and stored in *J (HOST pointer).
 * Two-array storage.  Synchronises the stream.
 */
int lb_outlet_flux(lb_lattice *lat, double *J);

/*
 * Gradient of the outlet mass flux J (lb_outlet_flux) of the state after
 * nsteps steps with respect to the per-site x-force: lb_grad_force_x with the
 * seed dJ/dS_N = c_ix at the fluid sites of the plane x = nx - 1 (built on the
 * GPU), plus the direct term dJ/dF_x = -1/2 at those sites.  grad:
 * caller-owned DEVICE array of N floats (site order), overwritten with the
 * complete dJ/dF_x.  J: HOST pointer receiving J of the final state, or NULL.
 * Same requirements, memory and synchronisation as lb_grad_force_x.
 */
int lb_grad_outlet_flux_x(lb_lattice *lat, int nsteps, int every, float *grad, double *J);

/* ---- batches of lattices ------------------------------------------------- */

/*
 * A batch holds `count` independent lattices ("domains") with their own
 * extents, relaxation times, solid flags and body forces, and advances all of
 * them together: one kernel launch per step covers every site of every domain
 * (the fused update of Section 3.1 applied to each domain exactly as
 * lb_step applies it to one lattice, with the same D3Q19 set, bounce-back,
 * periodic faces and Guo force).  Domains never exchange data.
 * Sites, population order, storage codecs and the raw-state format are those
 * of the single-lattice calls above, per domain.
 */
typedef struct lb_batch lb_batch;

/*
 * Create a batch.  dims: HOST int[3 * count], (nx, ny, nz) of domain d at
 * 3d..3d+2, each >= 1.  taus: HOST double[count], each > 0.5 or +INFINITY.
 * flags: NULL (every domain all fluid) or a HOST array of count pointers,
 * each NULL (all fluid) or nx*ny*nz bytes of 0 (fluid) / 1 (solid), copied.
 * storage: LB_F32, LB_F16S or LB_BF16S.  hip_stream: the hipStream_t on
 * which all of the batch's work is enqueued (borrowed, as in lb_create_ex;
 * NULL is the default stream).  autotune: 0 = the default launch
 * shape (16-byte vectors of population rows, storage blocks of 32 KiB per
 * population, one workgroup per tile); 1 = time every candidate shape (sites
 * per lane, storage block size, grid size, tile order, and for 4-byte vectors
 * a cap of 4 or 5 resident workgroups per compute unit) on this batch once
 * and keep the fastest (results are remembered for the rest of the process,
 * keyed by the codec and the domains' extents).  Every domain starts at rest
 * with zero force; every step counter is 0.  All device memory is allocated
 * here and owned by the batch.  Returns NULL on failure (lb_last_error()).
 */
lb_batch *lb_batch_create(int count, const int *dims, const double *taus, const uint8_t *const *flags, int storage,
                          void *hip_stream, int autotune);

/* Free every resource of the batch (after waiting for its stream).  NULL is a no-op. */
void lb_batch_destroy(lb_batch *b);

/* Uniform force density of domain d (d = -1: every domain); as lb_set_force.
 * Synchronises the batch's stream. */
int lb_batch_set_force(lb_batch *b, int d, double fx, double fy, double fz);

/* Equilibrium initial state of domain d from caller-owned DEVICE FP64 fields
 * (N and 3N doubles of that domain, NULL = 1 and 0); as lb_init_eq. */
int lb_batch_init_eq(lb_batch *b, int d, const double *rho, const double *u);

/* Enqueue n >= 0 steps of every domain (asynchronous, one kernel launch per
 * step for all domains).  A request of 64 or more steps runs as one captured
 * HIP graph of the whole request (at most 1024 steps per graph), kept and
 * replayed for the next request of the same length. */
int lb_batch_step(lb_batch *b, int n);

/* Density and velocity of domain d into caller-owned DEVICE buffers (N and
 * 3N floats of that domain, either may be NULL); as lb_macros.  Enqueued. */
int lb_batch_macros(lb_batch *b, int d, float *rho, float *u);

/* FP64 {mass, momentum x, y, z} of the fluid sites of domain d after each of
 * the last k steps (out: 4k doubles, oldest first); as lb_sums. */
int lb_batch_sums(lb_batch *b, int d, double *out, int k);

/* Raw state of domain d in storage format (19 planes of that domain's N
 * elements); as lb_get_f / lb_set_f.  Host copies synchronise. */
int lb_batch_get_f(lb_batch *b, int d, void *buf, size_t bytes, int where);
int lb_batch_set_f(lb_batch *b, int d, const void *buf, size_t bytes, int where);

/* Wait for all work enqueued on the batch's stream. */
int lb_batch_sync(lb_batch *b);

/* Steps taken by the batch (every domain takes the same steps); -1 for a bad handle. */
long long lb_batch_steps_done(lb_batch *b);

/*
 * Integer properties: key 0 = kernel variant (1 / 2 / 3 = 16- / 8- / 4-byte
 * vectors per lane and population), 1 = sites per lane, 2 = workgroups per
 * step launch, 3 = tiles of 256 lanes over all domains, 4 = tile order, 5 =
 * domains, 6 = sites of all domains, 7 = fluid sites of all domains, 8 =
 * bytes of both population arrays of all domains, 9 = target bytes of one
 * population in a storage block, 10 = grid multiple (0: one workgroup per
 * tile), 11 = 1 if the shape was chosen by the autotuner, 12 = cap on the
 * resident step workgroups per compute unit (0: none).  -1 on error.
 */
long long lb_batch_query(lb_batch *b, int key);

/* Measurement helpers, as lb_time_steps / lb_time_step_kernel (the state advances). */
int lb_batch_time_steps(lb_batch *b, int n, double *ms);
int lb_batch_time_step_kernel(lb_batch *b, int n, double *ms);

/* ---- two-dimensional D2Q9 lattices ---------------------------------------- */

/*
 * The paper's own model (Section 2: D2Q9, nine velocities; Section 3.3: the
 * lid-driven cavity) run by the same fused pull update: BGK relaxation with
 * the second-order equilibrium (Eq. 1-3), halfway bounce-back, periodic
 * faces, FP32 storage of f - w, FP64 totals per step.
 * Sites s = x + nx * y.  Populations (raw-state layout of lb2d_get_f):
 *   0 (0,0); 1 (+1,0); 2 (-1,0); 3 (0,+1); 4 (0,-1); 5 (+1,+1); 6 (+1,-1);
 *   7 (-1,+1); 8 (-1,-1).  Weights 4/9, 1/9, 1/36.
 */
typedef struct lb2d_lattice lb2d_lattice;

/*
 * Create an nx * ny lattice.  flags: HOST array of nx*ny bytes (copied) or
 * NULL; 0 fluid, 1 wall (no-slip, at rest), 2 lid (a wall moving with
 * velocity (lid_ux, lid_uy)): a population bounced off the lid gains
 * 6 w_i (c_i . u_lid) (a moving wall of density 1).  tau > 0.5 or +INFINITY.
 * hip_stream: borrowed, NULL = the default stream.  Starts at rest.
 * Returns NULL on failure (lb_last_error()).
 */
lb2d_lattice *lb2d_create(int nx, int ny, double tau, const uint8_t *flags, double lid_ux, double lid_uy,
                          void *hip_stream);
void lb2d_destroy(lb2d_lattice *lat);

/* Equilibrium initial state from caller-owned DEVICE FP64 rho (N) and u (2N, u_x then u_y); NULL = 1 / 0. */
int lb2d_init_eq(lb2d_lattice *lat, const double *rho, const double *u);

/* Enqueue n >= 0 steps. */
int lb2d_step(lb2d_lattice *lat, int n);

/* rho = sum f and u = sum c f / rho of the stored state into DEVICE rho (N) and u (2N); solid sites 0. */
int lb2d_macros(lb2d_lattice *lat, float *rho, float *u);

/* FP64 {mass, momentum x, y} of the fluid sites after each of the last k steps (out: 3k doubles). */
int lb2d_sums(lb2d_lattice *lat, double *out, int k);

/* Raw state: 9 planes of N floats (g = f - w), host or device (where). */
int lb2d_get_f(lb2d_lattice *lat, void *buf, size_t bytes, int where);
int lb2d_set_f(lb2d_lattice *lat, const void *buf, size_t bytes, int where);

int lb2d_sync(lb2d_lattice *lat);
long long lb2d_steps_done(lb2d_lattice *lat);

/* Milliseconds for n steps between two HIP events on the lattice's stream (the state advances). */
int lb2d_time_steps(lb2d_lattice *lat, int n, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* LB_H */
