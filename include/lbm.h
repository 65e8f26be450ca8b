/*
 * lbm.h -- C ABI of the MI355X (gfx950) cascaded central-moment D2Q9 lattice
 * Boltzmann library (liblbm.so).
 *
 * The method is the cascaded LBM with central-moment forcing of Ning &
 * Premnath, "Numerical Study of the Properties of the Central Moment Lattice
 * Boltzmann Method", Section II, with the boundary treatments of Section III
 * (periodic sides, halfway bounce-back walls, moving-wall bounce-back).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Every pointer argument named as a device buffer is device memory
 *   owned by the caller (the library never frees it); the library itself
 *   owns only the context and a small reduction scratch area allocated by
 *   the first lbm_diagnostics call (creating and destroying a context that
 *   never asks for diagnostics allocates no device memory).  Host pointers are named as such.
 * Streams.  All calls are asynchronous on the context's HIP stream, except
 *   lbm_diagnostics (synchronises that stream) and lbm_lattice_layout /
 *   lbm_create / lbm_destroy (host only).  A caller that reads a buffer on
 *   another stream must order it after the library's work itself.
 * Errors.  Every call returns an lbm_status and never aborts or throws.
 *   LBM_EINVAL: bad argument (message in lbm_last_error); nothing was
 *   launched.  LBM_EDEVICE: a HIP call or launch failed.  LBM_ESTATE: call
 *   out of order.  LBM_EUNSUPPORTED: valid request the context does not
 *   support (the adjoint with FP16/BF16 storage; the explicit-buffer step
 *   calls with stochastic rounding).  LBM_EUNSTABLE: the
 *   diagnostics found a non-finite sum.
 * Field types.  The "compute real" R of a context is double for LBM_FP64
 *   and float for every other storage mode.  Arrays that carry the state in
 *   or out -- initial fields (rho, ux, uy), populations, macroscopic outputs
 *   -- are FP64 in every mode: the library forms the deviations from the rest
 *   state in FP64 before narrowing, so an FP32 run is not limited by the
 *   ~6e-8 granularity of a float near rho0.  The force field, adjoint
 *   cotangents and gradients are in R.  Node fields are arrays [ny][nx]
 *   (x fastest, no padding); population arrays are [9][ny][nx].
 * Lattice.  A lattice buffer holds nine planes [9][ny][pitch] (x fastest,
 *   pitch = lbm_lattice_layout's pitch elements, a multiple of 64) of the
 *   storage type: double (LBM_FP64), float (LBM_FP32), IEEE binary16
 *   (LBM_FP16_DEV) or bfloat16 (LBM_BF16_DEV).  The stored value is the
 *   deviation f_a - w_a rho0 from the rest equilibrium (w = 4/9, 1/9 x4,
 *   1/36 x4), in every mode.  Buffers must be 256-byte aligned.
 * Time.  The state at time n is the pre-collision (post-streaming) f-bar(n)
 *   of Section II.  A lattice buffer holds the post-collision values of
 *   step n-1, i.e. the array from which pull streaming produces f-bar(n).
 *   lbm_init_equilibrium / lbm_set_populations set the state at time 0;
 *   every query returns the state at the current time.
 * Directions.  a = 0..8 in the order of Section II: e_x =
 *   (0,1,0,-1,0,1,-1,-1,1), e_y = (0,0,1,0,-1,1,1,-1,-1).
 */
#ifndef LBM_H_
#define LBM_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,
  LBM_EDEVICE = -2,
  LBM_ESTATE = -3,
  LBM_EUNSUPPORTED = -4,
  LBM_EUNSTABLE = -5
} lbm_status;

typedef enum {
  LBM_FP64 = 0,     /* double lattice, double arithmetic                    */
  LBM_FP32 = 1,     /* float lattice, float arithmetic                      */
  LBM_FP16_DEV = 2, /* binary16 deviations, float arithmetic                */
  LBM_BF16_DEV = 3  /* bfloat16 deviations, float arithmetic                */
} lbm_storage;

typedef enum {
  LBM_ROUND_NEAREST = 0,   /* round to nearest even                          */
  LBM_ROUND_STOCHASTIC = 1 /* unbiased stochastic rounding (16-bit modes)    */
} lbm_rounding;

typedef enum {
  LBM_PERIODIC = 0, /* wrap-around streaming (Sec. III, Poiseuille/Taylor-Green) */
  LBM_WALL = 1      /* halfway bounce-back wall, optionally moving tangentially
                       (Sec. III, Poiseuille walls and cavity lid)            */
} lbm_bc;

/* Problem statement of one lattice (Sec. II and III).
 *   nx, ny      fluid nodes; a wall sits half a spacing outside the first /
 *               last node (2 <= nx, ny; one plane, ny * pitch elements of
 *               the storage type, below 4 GiB).
 *   omega_nu    shear rate omega_4 = omega_5 = 1/tau, in (0, 2); kinematic
 *               viscosity nu = (1/omega_nu - 1/2)/3 (Sec. II).
 *   omega3      bulk rate omega_3; omega6, omega7, omega8 the third- and
 *               fourth-order rates; each in (0, 2); the paper uses 1.
 *   fx, fy      uniform body force (force per unit volume), used when no
 *               force field is bound.
 *   bc          x_lo, x_hi, y_lo, y_hi; periodic sides come in pairs.
 *   wall_u      tangential speed of each wall: y-velocity for x_lo/x_hi,
 *               x-velocity for y_lo/y_hi (the lid is y_hi with wall_u[3] =
 *               U).  A link crossing a moving wall receives
 *               6 rho0 w_a (e_a . U_wall) (Sec. III cavity).  A link
 *               crossing two walls passes through their corner point, taken
 *               at rest: plain bounce-back, no wall term.
 *   rho0        reference density (> 0): the deviation offset and the
 *               moving-wall density.
 *   storage     lbm_storage.
 *   rounding    LBM_ROUND_NEAREST (0): stores round to nearest even.
 *               LBM_ROUND_STOCHASTIC (1, FP16/BF16 only): each stored
 *               deviation is rounded up or down with probability
 *               proportional to its distance to the two neighbours
 *               (unbiased), the random bits drawn from a counter-based hash
 *               of (node, step, seed); deterministic for a given seed and
 *               bit-exact across restarts.  Lets slowly evolving flows
 *               progress whose change per step is below half an ulp of the
 *               16-bit format.
 *   seed        key of the stochastic-rounding hash. */
typedef struct {
  int32_t nx, ny;
  double omega_nu;
  double omega3, omega6, omega7, omega8;
  double fx, fy;
  int32_t bc[4];
  double wall_u[4];
  double rho0;
  int32_t storage;
  int32_t rounding;
  uint64_t seed;
} lbm_params;

typedef struct lbm_ctx lbm_ctx;

/* Lattice geometry for p: *pitch (elements per row, a multiple of 64) and
 * *bytes (size of one lattice buffer, 9 * ny * pitch * sizeof(storage)).
 * Host only. */
lbm_status lbm_lattice_layout(const lbm_params* p, int64_t* pitch, int64_t* bytes);

/* Create a context.  lat0 and lat1 are two lattice buffers (ping-pong;
 * lbm_lattice_layout bytes each).  force_field is NULL (uniform fx, fy) or a
 * device R array [2][ny][nx] (F_x plane then F_y plane), read by every step.
 * stream is a hipStream_t (NULL = default stream).  Validates p (EINVAL) and
 * allocates the context (host memory; EDEVICE on failure).  On success *out
 * owns it, and the scratch area it may allocate, until lbm_destroy.  The
 * state is undefined until lbm_init_equilibrium or lbm_set_populations.
 * Several contexts may share lat0/lat1 (each on its own stream, say); the
 * calls that take explicit buffers (lbm_step_sequence, lbm_step_between and
 * the adjoint calls) never touch a context's own lattices. */
lbm_status lbm_create(const lbm_params* p, void* lat0, void* lat1,
                      const void* force_field, void* stream, lbm_ctx** out);

/* Free the context (not the caller's buffers).  NULL is a no-op. */
void lbm_destroy(lbm_ctx* ctx);

/* Message of the last failed call on ctx, or of the last failed lbm_create
 * on this thread when ctx is NULL.  Valid until the next call. */
const char* lbm_last_error(const lbm_ctx* ctx);

/* Re-target the context to another hipStream_t. */
lbm_status lbm_set_stream(lbm_ctx* ctx, void* stream);

/* Number of steps taken since the state was last set. */
int64_t lbm_time(const lbm_ctx* ctx);

/* Device pointer of the lattice buffer holding the current state. */
void* lbm_current_lattice(const lbm_ctx* ctx);

/* Set the state at time 0 to f-bar = f^eq(rho, u) - S(u, F)/2: the
 * distribution whose central moments about u are the transformed equilibrium
 * (rho, -F_x/2, -F_y/2, rho/3, rho/3, 0, 0, 0, rho/9) of Sec. II, so that the
 * velocity of Sec. II's definition equals ux, uy exactly.  rho, ux, uy:
 * device FP64 arrays [ny][nx]. */
lbm_status lbm_init_equilibrium(lbm_ctx* ctx, const void* rho, const void* ux,
                                const void* uy);

/* Set the state at time 0 to arbitrary populations f-bar (device FP64
 * [9][ny][nx]); the deviations are rounded to the storage type. */
lbm_status lbm_set_populations(lbm_ctx* ctx, const void* f);

/* Write the current pre-collision populations f-bar(n) (device FP64
 * [9][ny][nx]). */
lbm_status lbm_get_populations(lbm_ctx* ctx, void* f);

/* Advance n >= 0 steps (Sec. II stream-and-collide: per node raw moments,
 * central moments about u, relaxation of each central moment at its own
 * rate with central-moment forcing, back to populations; pull streaming with
 * the boundary rules).  Steps are fused per kernel launch, four at a time
 * for LBM_FP64 and LBM_FP32 and two for the 16-bit modes, with the
 * intermediate states in on-chip memory; the result equals n single steps
 * bit for bit.  Ping-pong between lat0 and lat1. */
lbm_status lbm_step(lbm_ctx* ctx, int64_t n);

/* One step from lattice buffer src (state n) into dst (state n+1), outside
 * the ping-pong (used to recompute a segment of states for the adjoint).
 * src != dst; both lattice buffers of this context's layout.  Does not change
 * lbm_time or the current lattice.  LBM_EUNSUPPORTED for a context with
 * stochastic rounding: the call has no step index to key the random bits
 * by (lbm_step has one). */
lbm_status lbm_step_between(lbm_ctx* ctx, const void* src, void* dst);

/* n >= 0 single steps that keep every state: states[0] = step(src),
 * states[i] = step(states[i-1]).  states: host array of n device lattice
 * buffers of this context's layout, 256-byte aligned, none equal to its
 * input (src for states[0], states[i-1] for states[i]); a buffer may be
 * reused once its state has been read (ping-pong).  The segment recompute
 * of a checkpointed adjoint.  Same result as n calls of lbm_step_between
 * (groups of four steps whose five buffers are distinct may run as one
 * fused launch).  Does not change lbm_time or the current lattice.
 * LBM_EUNSUPPORTED for a context with stochastic rounding (as
 * lbm_step_between). */
lbm_status lbm_step_sequence(lbm_ctx* ctx, const void* src, void* const* states, int64_t n);

/* Copy the current lattice to dst (snapshot) / src to the current lattice
 * (restore; also sets lbm_time to t).  Device lattice buffers. */
lbm_status lbm_snapshot(lbm_ctx* ctx, void* dst);
lbm_status lbm_restore(lbm_ctx* ctx, const void* src, int64_t t);

/* Hydrodynamic fields of the current state (Sec. II): rho = sum f-bar,
 * u = (sum f-bar e + F/2)/rho, and the strain rate from the
 * non-equilibrium second moments (Sec. II, strain-rate relations, combined
 * for omega_3 != omega_4):
 *   d_x j_x = -3/4 (omega_3 f3neq + omega_4 f4neq),
 *   d_y j_y = -3/4 (omega_3 f3neq - omega_4 f4neq),
 *   d_x j_y + d_y j_x = -3 omega_5 f5neq,
 * sxx = d_x j_x / rho, syy = d_y j_y / rho, sxy = (d_x j_y + d_y j_x)/(2 rho).
 * Each output is a device FP64 array [ny][nx] or NULL (skipped). */
lbm_status lbm_macroscopic(lbm_ctx* ctx, void* rho, void* ux, void* uy,
                           void* sxx, void* syy, void* sxy);

/* Global sums of the current state, accumulated in FP64 with a fixed
 * reduction order (deterministic): out[0] = sum rho, out[1] = sum rho ux,
 * out[2] = sum rho uy, out[3] = 1/2 sum rho |u|^2 (host array of 4).
 * Synchronises the stream.  The first call on a context allocates its
 * reduction scratch area (33 KB of device memory; EDEVICE on failure).
 * Returns LBM_EUNSTABLE if any sum is not finite. */
lbm_status lbm_diagnostics(lbm_ctx* ctx, double out[4]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums of
 * lbm_diagnostics, with the same kernels and the same fixed reduction order
 * (equal bit for bit), written to out, a device FP64 array of 4 (8-byte
 * aligned) owned by the caller.  Asynchronous on the context's stream: no
 * synchronisation, no copy to the host, no finiteness check (the caller reads
 * out after the stream's work, and checks it).  The partial sums live in a
 * static device array of the library, 1024 x 4 doubles (32 KiB) per GPU, held
 * until the process ends; the call allocates nothing.  The need does not grow
 * with the lattice (the reduction grid is fixed at 1024 blocks); a context
 * whose grid exceeds the array is refused with LBM_EINVAL.  Every call on a
 * GPU shares that GPU's array: calls that overlap in time on one GPU (other
 * streams, other threads) race and must be ordered by the caller.  The first
 * call on a device looks up the array's device address (with that device
 * current).  LBM_ESTATE before the state is set; LBM_EDEVICE on a HIP
 * failure. */
lbm_status lbm_diagnostics_noalloc(lbm_ctx* ctx, void* out);

/* Adjoint (vector-Jacobian product) of one step n-1 -> n.  lat_prev: the
 * lattice buffer of state n-1 (as stored by the forward).  mu_in: cotangent
 * of the lattice buffer of state n, a device R array in lattice layout
 * [9][ny][pitch].  mu_out (!= mu_in): receives the cotangent of the buffer of
 * state n-1 (fully overwritten).  grad_force: NULL, or device R [2][ny][nx]
 * to which dL/dF of this step is ADDED (requires a bound force field).  The
 * step is re-gathered from lat_prev; its transposed Jacobian is applied per
 * node and the result is scattered by reverse streaming (a permutation, no
 * atomics).  LBM_EUNSUPPORTED for FP16/BF16 storage. */
lbm_status lbm_adjoint_step(lbm_ctx* ctx, const void* lat_prev, const void* mu_in,
                            void* mu_out, void* grad_force);

/* n >= 0 adjoint steps newest-first over one segment: states[0..n-1] are the
 * lattice buffers of states k, k+1, ..., k+n-1 (host array of device
 * pointers), mu_a holds the cotangent of state k+n on entry.  The steps run
 * fused, the intermediate cotangents staying in on-chip memory: in groups
 * of four per launch on FP32 lattices of at least 200 000 nodes (and at
 * least 128 x 64), then in pairs, an odd one alone; each launch ping-pongs
 * between mu_a and mu_b (distinct buffers in lattice layout).  On return *result_in_b (host int)
 * is 0 if the cotangent of state k is in mu_a and 1 if it is in mu_b; the
 * other buffer is scratch.  grad_force as for lbm_adjoint_step (every step
 * ADDS its term, in the same order as single calls).  Same result as n calls
 * of lbm_adjoint_step, bit for bit.  LBM_EUNSUPPORTED for FP16/BF16
 * storage. */
lbm_status lbm_adjoint_sequence(lbm_ctx* ctx, const void* const* states, int64_t n, void* mu_a,
                                void* mu_b, void* grad_force, int* result_in_b);

/* Adjoint of the macroscopic map at lattice buffer lat: given cotangents
 * g_rho, g_ux, g_uy (device R [ny][nx]; any may be NULL = 0) of rho, ux, uy,
 * writes the cotangent of lat to mu_out (lattice layout, overwritten) and
 * ADDS the direct term dL/dF = (g_ux, g_uy)/(2 rho) to grad_force (may be
 * NULL). */
lbm_status lbm_adjoint_macroscopic(lbm_ctx* ctx, const void* lat, const void* g_rho,
                                   const void* g_ux, const void* g_uy, void* mu_out,
                                   void* grad_force);

/* Adjoint of lbm_init_equilibrium: given the cotangent mu0 of the initial
 * lattice buffer (lattice layout), writes the cotangents of the initial
 * fields to g_rho, g_ux, g_uy (device R [ny][nx]; any may be NULL) and ADDS
 * the initial-state part of dL/dF to grad_force (may be NULL).  rho, ux, uy
 * are the FP64 fields lbm_init_equilibrium was given. */
lbm_status lbm_adjoint_init(lbm_ctx* ctx, const void* rho, const void* ux,
                            const void* uy, const void* mu0, void* g_rho,
                            void* g_ux, void* g_uy, void* grad_force);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H_ */
