// engine.h -- host-side pieces shared by the solver and the server: error text,
// argument validation, the per-solve scalars, and the per-shape executor that launches
// the pass sequence of one step for a batch of members.
#pragma once
#include <hip/hip_runtime.h>

#include "eifp.h"
#include "passes.h"

namespace eifp {

// thread-local error text behind eifp_last_error()
eifp_status fail(eifp_status st, const char* fmt, ...);
void clear_error();
const char* last_error();

#define EIFP_HIP_TRY(expr)                                                                                       \
    do {                                                                                                         \
        hipError_t e_ = (expr);                                                                                  \
        if (e_ != hipSuccess) return ::eifp::fail(EIFP_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

// sizes: even, >= 4, factors 2 and 3 only, at most 512
eifp_status validate_shape(int nx, int ny, int nz);
// finite domain with right > left, mu and eps positive and finite
eifp_status validate_problem(const eifp_domain* dom, double mu, double eps);
// tau finite
eifp_status validate_tau(double tau);

// Per-solve scalars of the fused pass, formed in FP64 (Alg. 2 step 2: kappa = tau /
// sqrt(mu eps); the sqrt(mu), sqrt(eps) scalings of step 4 as their ratios).
PropParams make_params(int nx, int ny, int nz, const eifp_domain& dom, double mu, double eps, double tau);

// Host image of one member descriptor; same layout as MemberDesc<T> for either T.
struct DescImage {
    void* state;
    void* work;
    double* partials;
    double* inv;
    const void* spec;
    PropParams pp;
};
static_assert(sizeof(DescImage) == sizeof(MemberDesc<double>), "descriptor layout");
static_assert(sizeof(DescImage) == sizeof(MemberDesc<float>), "descriptor layout");

// Executor for one grid shape and precision: twiddle tables (FP64-formed, rounded to the
// working type) and the launch sequence.  Owns only the tables.
struct Engine {
    Grid3 g{};
    eifp_precision prec = EIFP_FP64;
    size_t tsize = 8;
    long long ns = 0;
    void* twx = nullptr;
    void* twy = nullptr;
    void* twz = nullptr;
    int nparts = 0;  // partial records per member written by the fused pass
    int nrec = 0;    // record capacity of a member's partials buffer (partial_capacity)
    long long bytes = 0;

    // allocate the tables and form them on the device (enqueued on stream, which is then
    // synchronised)
    eifp_status init(int nx, int ny, int nz, eifp_precision p, hipStream_t stream = nullptr);
    void release();
    size_t state_bytes() const { return (size_t)6 * (size_t)ns * tsize; }
    // room for the extended record (INV_XPART doubles per workgroup)
    size_t partial_bytes() const { return (size_t)nrec * INV_XPART * sizeof(double); }

    // One step (mode Z_STEP: x, z, fused y, z^-1 with the finalize, x^-1) or a forward-only
    // evaluation of the invariants (mode Z_FORWARD, or Z_FORWARD_EXT for the extended
    // record: state -> work, nothing stored back),
    // for nm members described by the device array md.  ev: 7 events recorded around
    // the kernels (or null).  want_inv = false skips the invariant partial sums and the
    // finalize (a step between output points).
    eifp_status passes(int mode, const void* md, int nm, hipStream_t st, hipEvent_t* ev, bool want_inv = true) const;
    // nsteps steps (mode Z_STEP), 7 events per step in ev (or null); steps n >= inv_from
    // reduce the invariants (0: every step; nsteps: none).  combine_x (only with
    // work != state for every member): the x inverse of a step and the x forward of the
    // next run as one kernel, which reads the state once instead of twice.
    eifp_status steps(const void* md, int nm, long long nsteps, hipStream_t st, hipEvent_t* ev, long long inv_from,
                      bool combine_x) const;
    // unscaled forward transform of each member's state into its work buffer
    eifp_status forward_spectrum(const void* md, int nm, hipStream_t st) const;
    // Jump: each member's state becomes the exact flow over its tau of its anchored
    // spectrum (fused propagate + inverse y from spec into work == state, z^-1, x^-1),
    // with the invariants if want_inv.
    eifp_status jump(const void* md, int nm, hipStream_t st, bool want_inv = true) const;
};

// Partial records a member's buffer must hold for grid g: those of the fused pass, or
// one per packed x column when the grid steps with the plane pass, whichever is more
// (-1: unsupported size).
template <typename T>
int partial_capacity(const Grid3& g);

// Bytes of the twiddle table of length n: n entries exp(-2 pi i k / n), plus their
// rounding remainders for FP32 tables.
template <typename T>
constexpr size_t twiddle_table_bytes(int n) {
    return (size_t)n * TwParts<T>::value * sizeof(cpx<T>);
}
// Form that table at tw on the device (k_twiddles, enqueued on st).
template <typename T>
eifp_status launch_twiddles(cpx<T>* tw, int n, hipStream_t st);

// Widen / narrow n reals on the device (enqueued on st).
eifp_status convert_f32_to_f64(const void* in, void* out, long long n, hipStream_t st);
eifp_status convert_f64_to_f32(const void* in, void* out, long long n, hipStream_t st);

}  // namespace eifp
