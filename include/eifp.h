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
 *     never keeps them.  All device memory is owned by the library.
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
    EIFP_ERR_STATE = 6             /* call not valid in the solver's current state */
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
 * Returns after enqueueing; the work runs on the solver's stream.  nsteps = 0 is a
 * no-op.  Errors: INVALID_ARG (NULL solver, non-finite tau, nsteps < 0), DEVICE. */
eifp_status eifp_step(eifp_solver *s, double tau, long long nsteps);

/* Same as eifp_step, and also measures each pass with HIP events recorded on the
 * solver's stream around every kernel.  pass_ms[0..5] receive the summed durations in
 * milliseconds of: x-forward (real-to-complex), z-forward, fused y (forward,
 * propagator, invariant partials, inverse), z-inverse, x-inverse (complex-to-real),
 * invariant finalize.  Synchronises the
 * stream before returning.  Errors as eifp_step, plus INVALID_ARG for NULL pass_ms. */
eifp_status eifp_step_timed(eifp_solver *s, double tau, long long nsteps, double *pass_ms);

/* Invariants of the current state (Sec. 4).  Synchronises the solver's stream.  If no
 * step has run since init, they are computed by a forward-only transform of the
 * state (the state is not modified).  Errors: INVALID_ARG (NULL), NONFINITE (a
 * non-finite invariant: the state holds NaN/Inf), DEVICE. */
eifp_status eifp_invariants(eifp_solver *s, eifp_invariant_set *out);

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

#ifdef __cplusplus
}
#endif

#endif /* EIFP_H */
