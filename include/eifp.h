/*
 * eifp.h -- C ABI of the MI355X EI-FP library (libeifp.so).
 *
 * The library advances the 3-D Maxwell system (1.1) of Wang & Jiang, "Time exponential
 * integrator Fourier pseudospectral methods ... for three-dimensional Maxwell's
 * equations" (arXiv:2210.06232), on a periodic cuboid with the fully discrete scheme
 * of Definition 2.3 / Algorithm 2: each step transforms the six field components with
 * the 3-D DFT (Sec. 2.3), applies the exact mode-wise exponential propagator of
 * Propositions 2.1-2.2 for the step size, transforms back, and reduces the discrete
 * invariants of Sec. 4.  All of it runs in HIP kernels on one gfx950 GPU.
 *
 * Conventions shared by every call:
 *   - Field arrays are FP64, component-major [3][nz][ny][nx] with x fastest, i.e. the
 *     vector ordering of Sec. 2.2: H[c][l][k][j] = H_c(x_j, y_k, z_l) with the
 *     collocation points x_j = xl + j (xr - xl)/nx, j = 0..nx-1 (Sec. 2.2, Def. 2.3 step 1).
 *   - Grid sizes must be even (Sec. 2.2) and at least 4, with only the prime factors
 *     2 and 3; nx in {4,6,8,12,...,512}, ny and nz in {4,6,8,12,16,...,384,512}.
 *   - Every call returns an eifp_status; on failure eifp_last_error() gives a
 *     thread-local description.  No call throws or aborts.
 *   - Host pointers are only read during the call that receives them; the library
 *     never keeps them.  Device memory the library allocates is owned by it; the
 *     caller's device buffers (eifp_fields_device, eifp_step_noalloc) stay the
 *     caller's and are only used by the work that call enqueues.
 *   - One solver may be used by one host thread at a time.
 */
#ifndef EIFP_H
#define EIFP_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eifp_solver eifp_solver; /* opaque, owned by the library */

typedef enum {
    EIFP_OK = 0,
    EIFP_ERR_INVALID_ARG = 1,      /* bad size, domain, material constant, step, pointer */
    EIFP_ERR_UNSUPPORTED_SIZE = 2, /* even size >= 4 with a prime factor above 3, or above 512 */
    EIFP_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed */
    EIFP_ERR_DEVICE = 4,           /* a HIP call or kernel launch failed */
    EIFP_ERR_NONFINITE = 5,        /* NaN/Inf in the initial fields or in the invariants */
    EIFP_ERR_STATE = 6,            /* call not valid in the solver's current state */
    EIFP_ERR_CANCELLED = 7         /* server request ended by eifp_server_cancel */
} eifp_status;

typedef enum {
    EIFP_FP64 = 0, /* transforms and propagator in FP64 */
    EIFP_FP32 = 1  /* transforms and propagator in FP32; twiddles, phases and propagator
                      coefficients formed in FP64 and rounded; invariant sums in FP64 */
} eifp_precision;

/* Omega = [xl, xr] x [yl, yr] x [zl, zr] (problem (1.1)-(1.2)); requires xr > xl etc. */
typedef struct {
    double xl, xr, yl, yr, zl, zr;
} eifp_domain;

/* Discrete invariants of the current state (Sec. 4), with <u, v>_N the grid mean of
 * u v (Sec. 3).  Computed on the device from the half spectrum by Parseval's identity;
 * summed in FP64 in a fixed order, so repeated runs give identical bits. */
typedef struct {
    double t;             /* time of the state: sum over step calls of tau * nsteps */
    long long steps_done; /* steps taken since init */
    double energy;        /* E1 = mu/2 <H,H>_N + eps/2 <E,E>_N              (Thm 4.1) */
    double helicity;      /* H1 = <H,DH>_N/(2 eps) + <E,DE>_N/(2 mu)         (Thm 4.3) */
    double momentum[3];   /* M1 = <H, B_k E>_N for k = 1, 2, 3 (x, y, z)     (Thm 4.4) */
    double div_h_l2;      /* ||div~(mu H)||_N                                (Thm 4.6) */
    double div_e_l2;      /* ||div~(eps E)||_N                               (Thm 4.6) */
} eifp_invariant_set;

/* Further conserved quantities of Thms 4.1 and 4.3, and drift scales, for the current
 * state, computed on
 * the device from the spectrum (Parseval), with the time derivatives taken from the
 * semi-discrete system (2.4): d/dt H = -(1/mu) D E, d/dt E = (1/eps) D H.  The
 * remaining ones of those theorems are identities: E5 = E6 = 0 (D_k is skew) and
 * M2 = -M1 (Thm 4.4). */
typedef struct {
    double t;             /* as eifp_invariant_set */
    long long steps_done;
    double e2;            /* E2 = mu/2 <H_t,H_t>_N + eps/2 <E_t,E_t>_N              (Thm 4.1) */
    double e3[3];         /* E3 = mu/2 <D_k H,D_k H>_N + eps/2 <D_k E,D_k E>_N, k = x,y,z */
    double e4[3];         /* E4 = the same on H_t, E_t                                      */
    double h2;            /* H2 = <H_t,D H_t>_N/(2 eps) + <E_t,D E_t>_N/(2 mu)       (Thm 4.3) */
    /* Drift scales of the current state: Cauchy-Schwarz bounds of the invariants that can
     * be near zero, to measure their drift against (|I(t) - I(0)| / scale) instead of
     * against |I(0)|.  With Sigma' the Parseval sum over the spectrum (grid-mean
     * normalisation, as the invariants) and b the discrete wave vector:
     *   |H1|      <= scale_helicity   = Sigma' |b| (|H^|^2/(2 eps) + |E^|^2/(2 mu))
     *   |M1_k|    <= scale_momentum[k] = sqrt(Sigma' |H^|^2) sqrt(Sigma' b_k^2 |E^|^2)
     *   div_h_l2  <= scale_div_h      = mu sqrt(Sigma' |b|^2 |H^|^2)   (likewise eps, E) */
    double scale_helicity;
    double scale_momentum[3];
    double scale_div_h;
    double scale_div_e;
} eifp_invariant_ext_set;

/* Create a solver and load the initial values (Def. 2.3 step 2).
 *   out       receives the handle (set to NULL on failure)
 *   nx,ny,nz  grid sizes (see above)
 *   dom       domain; mu, eps > 0 and finite (the material constants of (1.1))
 *   prec      working precision of the transforms and the propagator
 *   H0, E0    host arrays of 3*nx*ny*nz doubles each, [3][nz][ny][nx]; copied
 *   hip_stream  a hipStream_t to enqueue all work on, or NULL for a stream owned by
 *               the solver.  A caller-supplied stream must outlive the solver.
 * Errors: INVALID_ARG (odd/small size, empty domain, mu or eps <= 0 or non-finite,
 * NULL pointers), UNSUPPORTED_SIZE, NONFINITE (NaN/Inf in H0 or E0), OUT_OF_MEMORY,
 * DEVICE. */
eifp_status eifp_init(eifp_solver **out, int nx, int ny, int nz, const eifp_domain *dom, double mu, double eps,
                      eifp_precision prec, const double *H0, const double *E0, void *hip_stream);

/* Enqueue nsteps time steps of size tau (Alg. 2 with t_end = tau, repeated): forward
 * 3-D transform, exact propagator, inverse transform, invariant reduction.  tau may
 * be negative or arbitrarily large (the scheme has no step-size restriction, Thm 3.4).
 * Returns after enqueueing; the work runs on the solver's stream.  The fields after the
 * last step are what eifp_fields reads; the intermediate states of one call are formed
 * (with the same rounding as separate calls: n steps in one call and n calls of one step
 * give the same bits) but not stored, and after a DEVICE error the fields and invariants
 * are undefined.  nsteps = 0 is a no-op.  Errors: INVALID_ARG (NULL solver, non-finite
 * tau, nsteps < 0), DEVICE. */
eifp_status eifp_step(eifp_solver *s, double tau, long long nsteps);

/* Anchor: store the spectrum of the current state (its forward 3-D transform, Def. 2.3
 * step 2) on the device as the starting point of later eifp_jump calls.  Allocates one
 * state-sized device buffer on first use.  Enqueued.  Errors: INVALID_ARG, OUT_OF_MEMORY,
 * DEVICE. */
eifp_status eifp_anchor(eifp_solver *s);

/* Same result as eifp_step(s, tau, nsteps) up to rounding, computed in one propagation
 * from the anchor: the scheme is the exact flow of the Fourier semi-discretisation over
 * any time span (Def. 2.3, Prop. 2.1; Alg. 2 takes t_end in one step), so the new state
 * is the inverse transform of the anchored spectrum propagated over
 * (t + tau * nsteps - t_anchor).  Rounding errors therefore do not accumulate with the
 * number of steps (one forward transform at the anchor, one propagation and inverse
 * transform per call).  Anchors the current state first if there is no valid anchor;
 * eifp_step invalidates the anchor.  Invariants are computed for the new state.  Errors:
 * as eifp_step, plus OUT_OF_MEMORY (first anchor). */
eifp_status eifp_jump(eifp_solver *s, double tau, long long nsteps);

/* Same as eifp_step, and also measures each pass with HIP events recorded on the
 * solver's stream around every kernel.  pass_ms[0..5] receive the summed durations in
 * milliseconds of: x-forward (real-to-complex; only the first step of the call has a
 * kernel of its own), z-forward, fused y (forward, propagator, invariant partials,
 * inverse), z-inverse (which also finalizes the invariants, in one extra workgroup),
 * x-inverse (complex-to-real; between two steps of the call one kernel does this
 * step's x-inverse and the next step's x-forward, and its time is counted here), and
 * the gap where a separate finalize would run (kept for layout; near zero).
 * Synchronises the stream before returning.  Errors as eifp_step, plus INVALID_ARG for
 * NULL pass_ms. */
eifp_status eifp_step_timed(eifp_solver *s, double tau, long long nsteps, double *pass_ms);

/* Invariants of the current state (Sec. 4).  Synchronises the solver's stream.  If no
 * step has run since init, they are computed by a forward-only transform of the
 * state (the state is not modified).  Errors: INVALID_ARG (NULL), NONFINITE (a
 * non-finite invariant: the state holds NaN/Inf), DEVICE. */
eifp_status eifp_invariants(eifp_solver *s, eifp_invariant_set *out);

/* Extended invariants (eifp_invariant_ext_set) of the current state, by a forward-only
 * transform of the state (not modified).  Synchronises.  Errors: INVALID_ARG (NULL),
 * NONFINITE, DEVICE. */
eifp_status eifp_invariants_ext(eifp_solver *s, eifp_invariant_ext_set *out);

/* Copy the current fields to caller-owned host arrays of 3*nx*ny*nz doubles each,
 * layout [3][nz][ny][nx] (Def. 2.3 step 4 output).  FP32 state is widened exactly.
 * Synchronises the stream.  Errors: INVALID_ARG (NULL), DEVICE. */
eifp_status eifp_fields(eifp_solver *s, double *H, double *E);

/* Copy the current fields to caller-owned device buffers (e.g. torch tensors) of
 * 3*nx*ny*nz elements each in out_prec (FP64 -> double, FP32 -> float), same layout.
 * Enqueued on the solver's stream; does not synchronise.  Errors: INVALID_ARG, DEVICE. */
eifp_status eifp_fields_device(eifp_solver *s, void *H, void *E, eifp_precision out_prec);

/* Diagnostic: the forward 3-D transform of the current state (Def. 2.3 step 2), as the
 * packed half spectrum the kernels work on, copied to a host array of
 * 6*nz*ny*(nx/2)*2 doubles: [6][kz][ky][kx][re,im] for kx = 0..nx/2-1, components
 * Hx, Hy, Hz, Ex, Ey, Ez.  Entry kx = 0 holds F(0,ky,kz) + i F(nx/2,ky,kz) where F is the
 * full 3-D DFT; entries kx >= 1 hold F(kx,ky,kz).  The state is not modified.
 * Synchronises.  Errors: INVALID_ARG, DEVICE. */
eifp_status eifp_spectrum(eifp_solver *s, double *out);

/* Block until all work enqueued on the solver's stream is done.  Errors: DEVICE. */
eifp_status eifp_sync(eifp_solver *s);

/* The hipStream_t the solver enqueues on (as void*); NULL for a NULL solver. */
void *eifp_stream(eifp_solver *s);

/* Bytes of device memory held by the solver (state, scratch, tables, partials). */
long long eifp_device_bytes(eifp_solver *s);

/* Release the solver and its device memory; NULL is accepted.  Synchronises first. */
eifp_status eifp_destroy(eifp_solver *s);

/* Static text for a status code. */
const char *eifp_status_string(eifp_status st);

/* Detail of the last failure on the calling thread ("" if none). */
const char *eifp_last_error(void);

/* ===================================================================================
 * Serving: a persistent loop that runs many independent solves of the scheme above
 * (each one an init + step(tau, nsteps) with invariants every `cadence` steps) as they
 * arrive.  Same-shape, same-precision solves share every kernel launch (a batch of
 * "members"); solves of different shapes run on separate streams and overlap on the
 * device.  Requests are admitted in arrival order as their device footprint fits the
 * memory budget and the batch has a free slot; new ones join a batch between chunks
 * of steps, so a request never waits for the whole batch to finish.  Each member's
 * arithmetic is independent of the others in its batch: a solve gives the same bits
 * alone and in any mix.  A request can be cancelled while queued or running; a failed
 * batch ends only its own members.
 *
 * Threading: every server call may be made from any host thread; one internal thread
 * drives the GPU.
 * =================================================================================== */
typedef struct eifp_server eifp_server; /* opaque, owned by the library */

enum {
    EIFP_SERVER_DRY_RUN = 1,  /* schedule only: no device memory, no kernels (host tests) */
    EIFP_SERVER_NO_GRAPHS = 2,/* launch kernels one by one instead of replaying a captured
                                 HIP graph per (shape, batch size) */
    EIFP_SERVER_SERIAL = 4    /* at most one solve on the device at a time (baseline) */
};

enum {
    EIFP_REQ_KEEP_RESULT = 1, /* keep the final fields on the device after completion,
                                 for eifp_server_fields, until eifp_server_release */
    EIFP_REQ_NO_SNAPSHOT = 2, /* no device-side field snapshot at each output */
    EIFP_REQ_ANCHORED = 4     /* compute each output by a jump from the stored spectrum of
                                 the initial state (as eifp_jump) instead of stepping:
                                 one propagation and inverse transform per output, no
                                 error accumulation; costs one more state-sized buffer */
};

/* One solve (Alg. 2 on Omega = dom with constants mu, eps, step tau, nsteps steps). */
typedef struct {
    int nx, ny, nz;             /* as eifp_init */
    eifp_domain dom;
    double mu, eps, tau;        /* tau finite, may be negative */
    long long nsteps;           /* >= 1 */
    long long cadence;          /* an output event every `cadence` steps; 0: only at the end */
    eifp_precision prec;
    const double *H0, *E0;      /* host, 3*nx*ny*nz doubles each, [3][nz][ny][nx]; copied by submit */
    unsigned long long user_tag;/* returned in every event of this request */
    int flags;                  /* EIFP_REQ_* */
} eifp_request;

typedef enum {
    EIFP_EV_OUTPUT = 0, /* cadence point reached: invariants after `step` steps */
    EIFP_EV_DONE = 1,   /* all steps done: final invariants */
    EIFP_EV_ERROR = 2   /* the request failed (status says why) and was dropped */
} eifp_event_kind;

typedef struct {
    unsigned long long user_tag;
    long long req_id;
    int kind;                   /* eifp_event_kind */
    eifp_status status;
    long long step;             /* steps done when the event was produced */
    eifp_invariant_set inv;     /* invariants of the state after `step` steps */
    double t_arrive;            /* seconds on the server's clock: submit */
    double t_admit;             /* admission (device memory allocated, upload enqueued) */
    double t_event;             /* the event was observed complete on the host */
} eifp_event;

typedef struct {
    long long submitted, admitted, completed, failed;
    long long queued, running;  /* now */
    long long peak_running;     /* most requests admitted at once */
    double p50_s, p99_s, mean_s, max_s; /* latency = completion - arrival, completed requests */
    double point_steps;         /* sum over completed requests of nx*ny*nz*nsteps */
    double wall_s;              /* first arrival -> last completion */
    double point_steps_per_s;   /* point_steps / wall_s */
    long long bytes_in_use, peak_bytes, budget_bytes;
    long long chunks;           /* batched chunk launches */
    double mean_batch;          /* members per chunk, averaged over chunks */
    long long cancelled;        /* requests ended by eifp_server_cancel (not in failed) */
} eifp_server_stat_set;

/* Create a server.
 *   hbm_budget_bytes  device memory the server may hold for solves (footprints below
 *                     plus per-batch tables); requests wait until theirs fits
 *   max_batch         members per batch (1..1024)
 *   flags             EIFP_SERVER_*
 * For tests of failure handling, the environment variable EIFP_SERVER_FAULT_CHUNK=n, if
 * set when the server is created, makes its n-th chunk (counted over all batches from 1)
 * fail as a device error would, before anything is enqueued: the members of that batch
 * end with an error event (status DEVICE) and their memory is returned; other requests
 * are not affected.
 * Errors: INVALID_ARG, DEVICE (stream or thread creation failed). */
eifp_status eifp_server_create(eifp_server **out, long long hbm_budget_bytes, int max_batch, int flags);

/* Device bytes one request of this shape holds while admitted: its state, plus an equal
 * snapshot buffer unless EIFP_REQ_NO_SNAPSHOT, plus an equal spectrum buffer with
 * EIFP_REQ_ANCHORED, plus, for a request without EIFP_REQ_ANCHORED whose state is 64 MiB
 * or more, an equal work buffer (its batches then run the x inverse of a step and the x
 * forward of the next as one kernel).  0 for an invalid shape or precision. */
long long eifp_server_footprint(int nx, int ny, int nz, eifp_precision prec, int flags);

/* Queue a solve; the fields are copied before returning.  *req_id receives its id.
 * Errors: INVALID_ARG (as eifp_init, plus nsteps < 1, cadence < 0), UNSUPPORTED_SIZE,
 * NONFINITE, OUT_OF_MEMORY (the footprint alone exceeds the budget), STATE (server
 * shutting down). */
eifp_status eifp_server_submit(eifp_server *sv, const eifp_request *rq, long long *req_id);

/* Take up to max_events events (oldest first) into ev; *n_events receives the count.
 * Waits up to wait_ms milliseconds for the first one (0: do not wait, < 0: wait until
 * one arrives or the server has no queued or running request).  Errors: INVALID_ARG. */
eifp_status eifp_server_poll(eifp_server *sv, eifp_event *ev, int max_events, int *n_events, int wait_ms);

/* Copy a request's fields to host arrays as eifp_fields: for a running request, its
 * latest snapshot (taken at an output point; it may be newer than the last event
 * polled); for a finished request kept with EIFP_REQ_KEEP_RESULT, its final state.
 * *step (if not NULL) receives the step count of the copied fields.  Blocks until the
 * copy is done.  Errors: INVALID_ARG (unknown id, NULL), STATE (no snapshot yet,
 * snapshots disabled, result not kept or released), DEVICE. */
eifp_status eifp_server_fields(eifp_server *sv, long long req_id, double *H, double *E, long long *step);

/* Free the device memory of a finished request kept with EIFP_REQ_KEEP_RESULT.
 * Errors: INVALID_ARG (unknown id), STATE (not finished or not kept). */
eifp_status eifp_server_release(eifp_server *sv, long long req_id);

/* Cancel a queued or running request.  A queued one is dropped at once; a running one
 * leaves its batch when the chunk in flight (if any) has completed and no
 * eifp_server_fields copy is reading it, so that no kernel or copy still uses its
 * memory when that memory is returned.  Either way its last event is an error event with
 * status CANCELLED (after any output events of steps already run), and the request
 * counts in `cancelled`, not in `failed`.  Its batch companions run on unaffected.
 * Cancelling again before that event is a no-op.
 * Errors: INVALID_ARG (NULL server, unknown id: never submitted or already ended without
 * a kept result), STATE (finished with a kept result: use eifp_server_release). */
eifp_status eifp_server_cancel(eifp_server *sv, long long req_id);

/* Counters and latency percentiles so far. */
eifp_status eifp_server_stats(eifp_server *sv, eifp_server_stat_set *out);

/* Block until no request is queued or running (or timeout_ms passes, if >= 0; then
 * STATE).  Errors: INVALID_ARG, STATE, DEVICE. */
eifp_status eifp_server_drain(eifp_server *sv, int timeout_ms);

/* Stop the loop, drop queued requests, wait for running chunks, free everything.
 * No other call on this server may be in progress when it is made, or follow it.
 * NULL is accepted. */
eifp_status eifp_server_destroy(eifp_server *sv);

/* ---------------------------------------------------------------------------------
 * Allocation-free stepping
 * ---------------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): eifp_step's time steps applied in
 * place to a caller-owned device state, with no solver object and no device allocation.
 * The library's own working data for the call (member descriptor, twiddle tables, the
 * fused pass's partial sums, the invariant record) lives in a fixed 4 MiB device array
 * that each GPU the library runs on holds until the process ends; every supported grid
 * fits in it, and a grid that would not is rejected with UNSUPPORTED_SIZE before anything
 * is enqueued.  The call only enqueues work (a set-up kernel, then the passes of each
 * step); it makes no hipMalloc/hipFree and does not synchronise.  All calls on one GPU
 * share that array: calls whose work overlaps on the device race and must be ordered by
 * the caller (one stream, or events).  Results equal eifp_init + eifp_step +
 * eifp_fields_device of the same fields, in the same precision.
 *   fields    device buffer, 16-byte aligned, of 6*nx*ny*nz elements of the working
 *             precision (double for EIFP_FP64, float for EIFP_FP32): Hx, Hy, Hz, Ex, Ey,
 *             Ez, each [nz][ny][nx] with x fastest; read and overwritten in place
 *   nx..prec  as eifp_init; tau, nsteps as eifp_step (nsteps = 0 enqueues nothing)
 *   inv_out   NULL, or a device buffer of 8 doubles that receives the invariants of the
 *             final state: E1, H1, M1x, M1y, M1z, ||div~(mu H)||_N, ||div~(eps E)||_N, 0
 *             (eifp_invariant_set's order; reduced on the last step only)
 *   hip_stream  the hipStream_t to enqueue on (NULL: the null stream)
 * Errors (all detected on the host before anything is enqueued): INVALID_ARG (NULL or
 * misaligned pointers, pointers that are not device memory or whose allocation is too
 * short, sizes, domain, mu, eps, tau, nsteps < 0, unknown precision), UNSUPPORTED_SIZE,
 * DEVICE (a failed launch). */
eifp_status eifp_step_noalloc(void *fields, int nx, int ny, int nz, const eifp_domain *dom, double mu, double eps,
                              eifp_precision prec, double tau, long long nsteps, double *inv_out, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* EIFP_H */
