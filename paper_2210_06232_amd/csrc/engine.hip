// engine.hip -- error text, validation, per-solve scalars and the per-shape executor.
#include "engine.h"

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

namespace eifp {

namespace {
thread_local std::string g_err;

bool only_2_3(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kPi = 3.141592653589793238462643383279502884;

template <typename T>
eifp_status make_table(void** dst, int n, long long* bytes, hipStream_t st) {
    const size_t nb = twiddle_table_bytes<T>(n);
    if (hipMalloc(dst, nb) != hipSuccess) {
        *dst = nullptr;
        (void)hipGetLastError();
        return fail(EIFP_ERR_OUT_OF_MEMORY, "twiddle table allocation failed");
    }
    *bytes += (long long)nb;
    return launch_twiddles<T>((cpx<T>*)*dst, n, st);
}

eifp_status rc_to_status(int rc, const char* what) {
    if (rc == kOk) return EIFP_OK;
    if (rc == kUnsupported) return fail(EIFP_ERR_UNSUPPORTED_SIZE, "%s: no compiled plan for this size", what);
    return fail(EIFP_ERR_DEVICE, "%s: kernel launch failed: %s", what, hipGetErrorString(hipGetLastError()));
}

// Grids whose (y, z) plane fits in LDS step with the plane pass in place of the z
// forward, fused y and z inverse passes (the partial records it writes, one per packed
// x column, must fit the member's partials buffer, which every caller sizes for
// partial_capacity records); the x kernel after it finalizes.
template <typename T>
bool use_plane(const Engine& en) {
    return plane_ok<T>(en.g) && en.g.M <= en.nrec;
}

}  // namespace

template <typename T>
int partial_capacity(const Grid3& g) {
    const int n = fused_partial_count<T>(AXIS_Y, g);
    if (n <= 0) return -1;
    return plane_ok<T>(g) && g.M > n ? g.M : n;
}
template int partial_capacity<double>(const Grid3&);
template int partial_capacity<float>(const Grid3&);

namespace {

// The middle of a plane step, between the x forward and the x inverse: events 2, 3, 4
// (the z slots empty, the fused slot holding the plane pass).
template <typename T>
eifp_status run_plane_middle(const Engine& en, const void* md, int nm, hipStream_t st, hipEvent_t* ev,
                             bool want_inv) {
    int rc;
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[2], st));
    if ((rc = launch_plane<T>(en.g, md, nm, en.twy, en.twz, want_inv ? 1 : 0, st))) return rc_to_status(rc, "plane pass");
    if (ev) {
        EIFP_HIP_TRY(hipEventRecord(ev[3], st));
        EIFP_HIP_TRY(hipEventRecord(ev[4], st));
    }
    return EIFP_OK;
}

template <typename T>
eifp_status run_passes(const Engine& en, int mode, const void* md, int nm, hipStream_t st, hipEvent_t* ev,
                       bool want_inv) {
    int rc;
    if (mode == Z_STEP && use_plane<T>(en)) {
        if (ev) EIFP_HIP_TRY(hipEventRecord(ev[0], st));
        if ((rc = launch_x<T>(X_FWD, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x forward");
        if (ev) EIFP_HIP_TRY(hipEventRecord(ev[1], st));
        eifp_status s = run_plane_middle<T>(en, md, nm, st, ev, want_inv);
        if (s) return s;
        if ((rc = launch_x<T>(X_INV, en.g, md, nm, en.twx, st, want_inv ? en.g.M : 0)))
            return rc_to_status(rc, "x inverse");
        if (ev) {
            EIFP_HIP_TRY(hipEventRecord(ev[5], st));
            EIFP_HIP_TRY(hipEventRecord(ev[6], st));
        }
        return EIFP_OK;
    }
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[0], st));
    if ((rc = launch_x<T>(X_FWD, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x forward");
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[1], st));
    if ((rc = launch_c2c<T>(false, AXIS_Z, en.g, md, nm, en.twz, st))) return rc_to_status(rc, "z forward");
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[2], st));
    if ((rc = launch_fused<T>(mode, AXIS_Y, en.g, md, nm, en.twy, want_inv ? 1 : 0, st)))
        return rc_to_status(rc, "fused y pass");
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[3], st));
    if (mode == Z_STEP) {
        // the z inverse also finalizes the invariant partials (one extra workgroup per member)
        if ((rc = launch_c2c<T>(true, AXIS_Z, en.g, md, nm, en.twz, st, want_inv ? en.nparts : 0)))
            return rc_to_status(rc, "z inverse");
        if (ev) EIFP_HIP_TRY(hipEventRecord(ev[4], st));
        if ((rc = launch_x<T>(X_INV, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x inverse");
        if (ev) EIFP_HIP_TRY(hipEventRecord(ev[5], st));
    } else if (ev) {
        EIFP_HIP_TRY(hipEventRecord(ev[4], st));
        EIFP_HIP_TRY(hipEventRecord(ev[5], st));
    }
    if (mode != Z_STEP && want_inv && (rc = launch_finalize<T>(md, nm, en.nparts, st, mode == Z_FORWARD_EXT)))
        return rc_to_status(rc, "finalize");
    if (ev) EIFP_HIP_TRY(hipEventRecord(ev[6], st));
    return EIFP_OK;
}

// nsteps steps; steps n >= inv_from reduce the invariants.  With work != state, the x
// inverse of each step but the last and the x forward of the step after it run as one
// kernel (X_INVFWD, in place on work: the state buffer is written by the last step
// only), and the z forward pass after it takes the components in ascending order.
// Events per step as in run_passes (the x forward slot is empty after the first step;
// the x inverse slot holds the combined kernel).  Grids with a plane pass run it in
// place of the three middle passes (use_plane).
template <typename T>
eifp_status run_steps(const Engine& en, const void* md, int nm, long long nsteps, hipStream_t st, hipEvent_t* ev,
                      long long inv_from, bool combine_x) {
    int rc;
    const bool plane = use_plane<T>(en);
    for (long long n = 0; n < nsteps; ++n) {
        const bool want_inv = n >= inv_from;
        hipEvent_t* e = ev ? ev + 7 * n : nullptr;
        const bool first = n == 0 || !combine_x, last = n + 1 == nsteps || !combine_x;
        if (e) EIFP_HIP_TRY(hipEventRecord(e[0], st));
        if (first && (rc = launch_x<T>(X_FWD, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x forward");
        if (e) EIFP_HIP_TRY(hipEventRecord(e[1], st));
        if (plane) {
            eifp_status s = run_plane_middle<T>(en, md, nm, st, e, want_inv);
            if (s) return s;
            if ((rc = launch_x<T>(last ? X_INV : X_INVFWD, en.g, md, nm, en.twx, st, want_inv ? en.g.M : 0)))
                return rc_to_status(rc, "x inverse");
            if (e) {
                EIFP_HIP_TRY(hipEventRecord(e[5], st));
                EIFP_HIP_TRY(hipEventRecord(e[6], st));
            }
            continue;
        }
        if ((rc = launch_c2c<T>(false, AXIS_Z, en.g, md, nm, en.twz, st, 0, first ? 1 : 0)))
            return rc_to_status(rc, "z forward");
        if (e) EIFP_HIP_TRY(hipEventRecord(e[2], st));
        if ((rc = launch_fused<T>(Z_STEP, AXIS_Y, en.g, md, nm, en.twy, want_inv ? 1 : 0, st)))
            return rc_to_status(rc, "fused y pass");
        if (e) EIFP_HIP_TRY(hipEventRecord(e[3], st));
        if ((rc = launch_c2c<T>(true, AXIS_Z, en.g, md, nm, en.twz, st, want_inv ? en.nparts : 0)))
            return rc_to_status(rc, "z inverse");
        if (e) EIFP_HIP_TRY(hipEventRecord(e[4], st));
        if ((rc = launch_x<T>(last ? X_INV : X_INVFWD, en.g, md, nm, en.twx, st)))
            return rc_to_status(rc, "x inverse");
        if (e) {
            EIFP_HIP_TRY(hipEventRecord(e[5], st));
            EIFP_HIP_TRY(hipEventRecord(e[6], st));
        }
    }
    return EIFP_OK;
}

template <typename T>
eifp_status run_spectrum(const Engine& en, const void* md, int nm, hipStream_t st) {
    int rc;
    if ((rc = launch_x<T>(X_FWD, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x forward");
    if ((rc = launch_c2c<T>(false, AXIS_Z, en.g, md, nm, en.twz, st))) return rc_to_status(rc, "z forward");
    if ((rc = launch_c2c<T>(false, AXIS_Y, en.g, md, nm, en.twy, st))) return rc_to_status(rc, "y forward");
    return EIFP_OK;
}

template <typename T>
eifp_status run_jump(const Engine& en, const void* md, int nm, hipStream_t st, bool want_inv) {
    int rc;
    if ((rc = launch_fused<T>(Z_JUMP, AXIS_Y, en.g, md, nm, en.twy, want_inv ? 1 : 0, st)))
        return rc_to_status(rc, "fused jump pass");
    if ((rc = launch_c2c<T>(true, AXIS_Z, en.g, md, nm, en.twz, st, want_inv ? en.nparts : 0)))
        return rc_to_status(rc, "z inverse");
    if ((rc = launch_x<T>(X_INV, en.g, md, nm, en.twx, st))) return rc_to_status(rc, "x inverse");
    return EIFP_OK;
}

template <typename TO, typename TI>
eifp_status convert(const void* in, void* out, long long n, hipStream_t st) {
    const long long blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536);
    hipLaunchKernelGGL((k_convert<TO, TI>), dim3(grid), dim3(256), 0, st, (const TI*)in, (TO*)out, (long)n);
    if (hipGetLastError() != hipSuccess) return fail(EIFP_ERR_DEVICE, "conversion kernel launch failed");
    return EIFP_OK;
}

}  // namespace

eifp_status fail(eifp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

void clear_error() { g_err.clear(); }

const char* last_error() { return g_err.c_str(); }

eifp_status validate_shape(int nx, int ny, int nz) {
    const int n3[3] = {nx, ny, nz};
    for (int w = 0; w < 3; ++w) {
        if (n3[w] < 4 || n3[w] % 2) return fail(EIFP_ERR_INVALID_ARG, "grid size %d must be even and >= 4", n3[w]);
        if (!only_2_3(n3[w]) || n3[w] > 512)
            return fail(EIFP_ERR_UNSUPPORTED_SIZE, "grid size %d: only 2^a 3^b up to 512 are supported", n3[w]);
    }
    return EIFP_OK;
}

eifp_status validate_problem(const eifp_domain* dom, double mu, double eps) {
    if (!dom) return fail(EIFP_ERR_INVALID_ARG, "NULL domain");
    const double lo[3] = {dom->xl, dom->yl, dom->zl}, hi[3] = {dom->xr, dom->yr, dom->zr};
    for (int w = 0; w < 3; ++w)
        if (!std::isfinite(lo[w]) || !std::isfinite(hi[w]) || !(hi[w] > lo[w]))
            return fail(EIFP_ERR_INVALID_ARG, "domain axis %d: need finite bounds with right > left", w);
    if (!(mu > 0) || !(eps > 0) || !std::isfinite(mu) || !std::isfinite(eps))
        return fail(EIFP_ERR_INVALID_ARG, "mu and eps must be positive and finite");
    return EIFP_OK;
}

eifp_status validate_tau(double tau) {
    if (!std::isfinite(tau)) return fail(EIFP_ERR_INVALID_ARG, "tau must be finite");
    return EIFP_OK;
}

PropParams make_params(int nx, int ny, int nz, const eifp_domain& dom, double mu, double eps, double tau) {
    PropParams pp;
    pp.tau_s = tau / std::sqrt(mu * eps);
    pp.tau_s_over_pi = pp.tau_s / kPi;
    pp.rh = std::sqrt(mu / eps);
    pp.re = std::sqrt(eps / mu);
    pp.inv_ns = 1.0 / ((double)nx * (double)ny * (double)nz);
    pp.nu[0] = kTwoPi / (dom.xr - dom.xl);
    pp.nu[1] = kTwoPi / (dom.yr - dom.yl);
    pp.nu[2] = kTwoPi / (dom.zr - dom.zl);
    pp.mu = mu;
    pp.eps = eps;
    pp.inv_mu = 1.0 / mu;
    pp.inv_eps = 1.0 / eps;
    return pp;
}

eifp_status Engine::init(int nx, int ny, int nz, eifp_precision p, hipStream_t stream) {
    g = Grid3{nx, ny, nz, nx / 2};
    prec = p;
    tsize = p == EIFP_FP64 ? 8 : 4;
    ns = (long long)nx * ny * nz;
    nparts = p == EIFP_FP64 ? fused_partial_count<double>(AXIS_Y, g) : fused_partial_count<float>(AXIS_Y, g);
    if (nparts <= 0) return fail(EIFP_ERR_UNSUPPORTED_SIZE, "no compiled plan for ny = %d", ny);
    nrec = p == EIFP_FP64 ? partial_capacity<double>(g) : partial_capacity<float>(g);
    eifp_status st = EIFP_OK;
    if (p == EIFP_FP64) {
        if ((st = make_table<double>(&twx, nx, &bytes, stream)) || (st = make_table<double>(&twy, ny, &bytes, stream)) ||
            (st = make_table<double>(&twz, nz, &bytes, stream)))
            return st;
    } else {
        if ((st = make_table<float>(&twx, nx, &bytes, stream)) || (st = make_table<float>(&twy, ny, &bytes, stream)) ||
            (st = make_table<float>(&twz, nz, &bytes, stream)))
            return st;
    }
    EIFP_HIP_TRY(hipStreamSynchronize(stream));
    return EIFP_OK;
}

void Engine::release() {
    for (void* q : {twx, twy, twz})
        if (q) (void)hipFree(q);
    twx = twy = twz = nullptr;
}

eifp_status Engine::passes(int mode, const void* md, int nm, hipStream_t st, hipEvent_t* ev, bool want_inv) const {
    return prec == EIFP_FP64 ? run_passes<double>(*this, mode, md, nm, st, ev, want_inv)
                             : run_passes<float>(*this, mode, md, nm, st, ev, want_inv);
}

eifp_status Engine::forward_spectrum(const void* md, int nm, hipStream_t st) const {
    return prec == EIFP_FP64 ? run_spectrum<double>(*this, md, nm, st) : run_spectrum<float>(*this, md, nm, st);
}

eifp_status Engine::steps(const void* md, int nm, long long nsteps, hipStream_t st, hipEvent_t* ev,
                          long long inv_from, bool combine_x) const {
    return prec == EIFP_FP64 ? run_steps<double>(*this, md, nm, nsteps, st, ev, inv_from, combine_x)
                             : run_steps<float>(*this, md, nm, nsteps, st, ev, inv_from, combine_x);
}

eifp_status Engine::jump(const void* md, int nm, hipStream_t st, bool want_inv) const {
    return prec == EIFP_FP64 ? run_jump<double>(*this, md, nm, st, want_inv)
                             : run_jump<float>(*this, md, nm, st, want_inv);
}

template <typename T>
eifp_status launch_twiddles(cpx<T>* tw, int n, hipStream_t st) {
    const int blocks = (n + 255) / 256;
    hipLaunchKernelGGL((k_twiddles<T>), dim3(blocks > 0 ? blocks : 1), dim3(256), 0, st, tw, n);
    if (hipGetLastError() != hipSuccess) return fail(EIFP_ERR_DEVICE, "twiddle table kernel launch failed");
    return EIFP_OK;
}
template eifp_status launch_twiddles<double>(cpx<double>*, int, hipStream_t);
template eifp_status launch_twiddles<float>(cpx<float>*, int, hipStream_t);

eifp_status convert_f32_to_f64(const void* in, void* out, long long n, hipStream_t st) {
    return convert<double, float>(in, out, n, st);
}

eifp_status convert_f64_to_f32(const void* in, void* out, long long n, hipStream_t st) {
    return convert<float, double>(in, out, n, st);
}

}  // namespace eifp
