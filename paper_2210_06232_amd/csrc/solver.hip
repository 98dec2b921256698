// solver.hip -- the EI-FP solver object and the C ABI declared in include/eifp.h.
//
// One step (Def. 2.3 / Alg. 2 with t_end = tau) is five kernels on the solver's stream:
//   x-forward (R2C split)  ->  y-forward  ->  fused z (forward, propagator, invariant
//   partials, inverse)  ->  y-inverse  ->  x-inverse (C2R merge)
// followed by a one-workgroup finalize of the invariant partials.  The state stays in
// HBM in the ABI's own layout ([6][nz][ny][nx] reals); all transforms are in place.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "eifp.h"
#include "passes.h"

using namespace eifp;

namespace {

thread_local std::string g_err;

eifp_status fail(eifp_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIP_TRY(expr)                                                                                      \
    do {                                                                                                   \
        hipError_t e_ = (expr);                                                                            \
        if (e_ != hipSuccess) return fail(EIFP_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool only_2_3(int n) {
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    return n == 1;
}

}  // namespace

// ---------------------------------------------------------------------------------
// deterministic compensated finalize (one workgroup)
// ---------------------------------------------------------------------------------
namespace eifp {

__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Thread j sums records j, j + 1024, ... (each record: INV_NPART contiguous doubles)
// with Neumaier compensation, then the 1024 (sum, compensation) pairs are combined by a
// fixed xor-butterfly inside each wave and a fixed loop over the 16 waves: the same
// partials always give the same bits.
__global__ void __launch_bounds__(1024) k_finalize(const double* __restrict__ partials, int nparts,
                                                   double* __restrict__ out) {
    __shared__ double s_w[16][2 * INV_NPART];
    double s[INV_NPART], c[INV_NPART];
#pragma unroll
    for (int q = 0; q < INV_NPART; ++q) s[q] = c[q] = 0.0;
    for (int j = threadIdx.x; j < nparts; j += 1024) {
        const double* rec = partials + (long)j * INV_NPART;
#pragma unroll
        for (int q = 0; q < INV_NPART; ++q) neumaier_add(s[q], c[q], rec[q]);
    }
#pragma unroll
    for (int q = 0; q < INV_NPART; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double os = __shfl_xor(s[q], off, 64), oc = __shfl_xor(c[q], off, 64);
            c[q] += oc;
            neumaier_add(s[q], c[q], os);
        }
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < INV_NPART; ++q) {
            s_w[wid][q] = s[q];
            s_w[wid][INV_NPART + q] = c[q];
        }
    }
    __syncthreads();
    double res[INV_NPART];
#pragma unroll
    for (int q = 0; q < INV_NPART; ++q) {
        double a = 0.0, ca = 0.0;
        for (int w = 0; w < 16; ++w) {
            ca += s_w[w][INV_NPART + q];
            neumaier_add(a, ca, s_w[w][q]);
        }
        res[q] = a + ca;
    }
    if (threadIdx.x == 0) {
        out[0] = res[INV_E1];
        out[1] = res[INV_H1];
        out[2] = res[INV_M1X];
        out[3] = res[INV_M1Y];
        out[4] = res[INV_M1Z];
        out[5] = sqrt(res[INV_DIVH]);
        out[6] = sqrt(res[INV_DIVE]);
        out[7] = 0.0;
    }
}

}  // namespace eifp

// ---------------------------------------------------------------------------------
// solver
// ---------------------------------------------------------------------------------
struct eifp_solver {
    int nx = 0, ny = 0, nz = 0, M = 0;
    long long ns = 0;
    eifp_domain dom{};
    double mu = 1, eps = 1;
    eifp_precision prec = EIFP_FP64;
    size_t tsize = 8;  // bytes per real in the working precision
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* state = nullptr;
    void* scratch = nullptr;
    void* twx = nullptr;
    void* twy = nullptr;
    void* twz = nullptr;
    double* partials = nullptr;
    int nparts = 0;
    double* inv_dev = nullptr;
    double* inv_host = nullptr;  // pinned
    bool inv_current = false;    // inv_dev describes the current state
    double t = 0.0;
    long long steps = 0;
    long long bytes = 0;
    std::vector<hipEvent_t> events;

    size_t state_bytes() const { return (size_t)6 * (size_t)ns * tsize; }
};

namespace {

template <typename T>
int upload_table(void** dst, int n, long long* bytes) {
    // exp(-2 pi i k / n), k < n, formed in FP64 and rounded to T
    std::vector<T> h(2 * (size_t)n);
    const double two_pi = 6.283185307179586476925286766559;
    for (int k = 0; k < n; ++k) {
        const double a = two_pi * (double)k / (double)n;
        h[2 * k] = (T)std::cos(a);
        h[2 * k + 1] = (T)-std::sin(a);
    }
    if (hipMalloc(dst, h.size() * sizeof(T)) != hipSuccess) return 1;
    *bytes += (long long)(h.size() * sizeof(T));
    if (hipMemcpy(*dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) return 2;
    return 0;
}

PropParams make_params(const eifp_solver* s, double tau) {
    PropParams pp;
    pp.tau_s = tau / std::sqrt(s->mu * s->eps);
    pp.rh = std::sqrt(s->mu / s->eps);
    pp.re = std::sqrt(s->eps / s->mu);
    pp.inv_ns = 1.0 / (double)s->ns;
    const double two_pi = 6.283185307179586476925286766559;
    pp.nu[0] = two_pi / (s->dom.xr - s->dom.xl);
    pp.nu[1] = two_pi / (s->dom.yr - s->dom.yl);
    pp.nu[2] = two_pi / (s->dom.zr - s->dom.zl);
    pp.mu = s->mu;
    pp.eps = s->eps;
    pp.inv_mu = 1.0 / s->mu;
    pp.inv_eps = 1.0 / s->eps;
    return pp;
}

eifp_status rc_to_status(int rc, const char* what) {
    if (rc == kOk) return EIFP_OK;
    if (rc == kUnsupported) return fail(EIFP_ERR_UNSUPPORTED_SIZE, "%s: no compiled plan for this size", what);
    return fail(EIFP_ERR_DEVICE, "%s: kernel launch failed: %s", what, hipGetErrorString(hipGetLastError()));
}

// The five passes of one step (or of the forward half when mode == Z_FORWARD, which
// reads src and leaves the spectrum in dst without touching src).
template <typename T>
eifp_status run_passes(eifp_solver* s, int mode, void* src, void* dst, double tau, hipEvent_t* ev) {
    const long rows = 6L * s->nz * s->ny;
    const long cs = (long)s->nz * s->ny * s->M;
    const PropParams pp = make_params(s, tau);
    int rc;
    if (ev) HIP_TRY(hipEventRecord(ev[0], s->stream));
    if ((rc = launch_x<T>(false, s->nx, src, dst, rows, s->twx, s->stream))) return rc_to_status(rc, "x forward");
    if (ev) HIP_TRY(hipEventRecord(ev[1], s->stream));
    if ((rc = launch_y<T>(false, s->ny, dst, s->M, s->nz, s->twy, s->stream))) return rc_to_status(rc, "y forward");
    if (ev) HIP_TRY(hipEventRecord(ev[2], s->stream));
    if ((rc = launch_z<T>(mode, s->nz, dst, s->M, s->ny, cs, s->twz, pp, s->partials, 1, s->stream)))
        return rc_to_status(rc, "z pass");
    if (ev) HIP_TRY(hipEventRecord(ev[3], s->stream));
    if (mode == Z_STEP) {
        if ((rc = launch_y<T>(true, s->ny, dst, s->M, s->nz, s->twy, s->stream))) return rc_to_status(rc, "y inverse");
        if (ev) HIP_TRY(hipEventRecord(ev[4], s->stream));
        if ((rc = launch_x<T>(true, s->nx, dst, dst, rows, s->twx, s->stream))) return rc_to_status(rc, "x inverse");
        if (ev) HIP_TRY(hipEventRecord(ev[5], s->stream));
    }
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(1024), 0, s->stream, (const double*)s->partials, s->nparts,
                       s->inv_dev);
    if (hipGetLastError() != hipSuccess) return fail(EIFP_ERR_DEVICE, "finalize launch failed");
    if (ev) HIP_TRY(hipEventRecord(ev[6], s->stream));
    return EIFP_OK;
}

eifp_status passes(eifp_solver* s, int mode, void* src, void* dst, double tau, hipEvent_t* ev) {
    return s->prec == EIFP_FP64 ? run_passes<double>(s, mode, src, dst, tau, ev)
                                : run_passes<float>(s, mode, src, dst, tau, ev);
}

template <typename TO, typename TI>
eifp_status convert(const void* in, void* out, long long n, hipStream_t st) {
    const long long blocks = (n + 255) / 256;
    const unsigned grid = (unsigned)(blocks < 65536 ? (blocks > 0 ? blocks : 1) : 65536);
    hipLaunchKernelGGL((k_convert<TO, TI>), dim3(grid), dim3(256), 0, st, (const TI*)in, (TO*)out, (long)n);
    if (hipGetLastError() != hipSuccess) return fail(EIFP_ERR_DEVICE, "conversion kernel launch failed");
    return EIFP_OK;
}

void release(eifp_solver* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void* p : {s->state, s->scratch, s->twx, s->twy, s->twz, (void*)s->partials, (void*)s->inv_dev})
        if (p) (void)hipFree(p);
    if (s->inv_host) (void)hipHostFree(s->inv_host);
    for (hipEvent_t e : s->events) (void)hipEventDestroy(e);
    if (s->own_stream && s->stream) (void)hipStreamDestroy(s->stream);
    delete s;
}

eifp_status alloc(void** p, size_t n, long long* bytes) {
    if (hipMalloc(p, n) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(EIFP_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed", n);
    }
    *bytes += (long long)n;
    return EIFP_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------------
extern "C" {

eifp_status eifp_init(eifp_solver** out, int nx, int ny, int nz, const eifp_domain* dom, double mu, double eps,
                      eifp_precision prec, const double* H0, const double* E0, void* hip_stream) {
    g_err.clear();
    if (!out) return fail(EIFP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!dom || !H0 || !E0) return fail(EIFP_ERR_INVALID_ARG, "NULL domain or field pointer");
    const int n3[3] = {nx, ny, nz};
    for (int w = 0; w < 3; ++w) {
        if (n3[w] < 4 || n3[w] % 2) return fail(EIFP_ERR_INVALID_ARG, "grid size %d must be even and >= 4", n3[w]);
        if (!only_2_3(n3[w]) || n3[w] > 512)
            return fail(EIFP_ERR_UNSUPPORTED_SIZE, "grid size %d: only 2^a 3^b up to 512 are supported", n3[w]);
    }
    const double lo[3] = {dom->xl, dom->yl, dom->zl}, hi[3] = {dom->xr, dom->yr, dom->zr};
    for (int w = 0; w < 3; ++w)
        if (!std::isfinite(lo[w]) || !std::isfinite(hi[w]) || !(hi[w] > lo[w]))
            return fail(EIFP_ERR_INVALID_ARG, "domain axis %d: need finite bounds with right > left", w);
    if (!(mu > 0) || !(eps > 0) || !std::isfinite(mu) || !std::isfinite(eps))
        return fail(EIFP_ERR_INVALID_ARG, "mu and eps must be positive and finite");
    if (prec != EIFP_FP64 && prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    const long long ns = (long long)nx * ny * nz;
    for (long long q = 0; q < 3 * ns; ++q)
        if (!std::isfinite(H0[q]) || !std::isfinite(E0[q]))
            return fail(EIFP_ERR_NONFINITE, "initial field holds NaN/Inf at flat index %lld", q);

    eifp_solver* s = new (std::nothrow) eifp_solver;
    if (!s) return fail(EIFP_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->nx = nx;
    s->ny = ny;
    s->nz = nz;
    s->M = nx / 2;
    s->ns = ns;
    s->dom = *dom;
    s->mu = mu;
    s->eps = eps;
    s->prec = prec;
    s->tsize = prec == EIFP_FP64 ? 8 : 4;
    eifp_status st = EIFP_OK;
#define INIT_TRY(expr)            \
    do {                          \
        st = (expr);              \
        if (st != EIFP_OK) {      \
            release(s);           \
            return st;            \
        }                         \
    } while (0)
#define INIT_HIP(expr)                                                                                      \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess) {                                                                             \
            release(s);                                                                                     \
            return fail(EIFP_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));                    \
        }                                                                                                   \
    } while (0)
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        INIT_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    const size_t sb = s->state_bytes();
    INIT_TRY(alloc(&s->state, sb, &s->bytes));
    INIT_TRY(alloc(&s->scratch, sb, &s->bytes));
    s->nparts = prec == EIFP_FP64 ? z_partial_count<double>(nz, s->M, ny) : z_partial_count<float>(nz, s->M, ny);
    if (s->nparts <= 0) {
        release(s);
        return fail(EIFP_ERR_UNSUPPORTED_SIZE, "no compiled z plan for nz = %d", nz);
    }
    INIT_TRY(alloc((void**)&s->partials, (size_t)s->nparts * INV_NPART * sizeof(double), &s->bytes));
    INIT_TRY(alloc((void**)&s->inv_dev, 8 * sizeof(double), &s->bytes));
    INIT_HIP(hipHostMalloc((void**)&s->inv_host, 8 * sizeof(double), hipHostMallocDefault));
    int trc = 0;
    if (prec == EIFP_FP64)
        trc = upload_table<double>(&s->twx, nx, &s->bytes) || upload_table<double>(&s->twy, ny, &s->bytes) ||
              upload_table<double>(&s->twz, nz, &s->bytes);
    else
        trc = upload_table<float>(&s->twx, nx, &s->bytes) || upload_table<float>(&s->twy, ny, &s->bytes) ||
              upload_table<float>(&s->twz, nz, &s->bytes);
    if (trc) {
        release(s);
        return fail(EIFP_ERR_OUT_OF_MEMORY, "twiddle table upload failed");
    }
    // upload: FP64 directly; FP32 through the scratch buffer (3 ns doubles = 6 ns floats)
    const size_t half = (size_t)3 * ns * sizeof(double);
    if (prec == EIFP_FP64) {
        INIT_HIP(hipMemcpyAsync(s->state, H0, half, hipMemcpyHostToDevice, s->stream));
        INIT_HIP(hipMemcpyAsync((char*)s->state + half, E0, half, hipMemcpyHostToDevice, s->stream));
    } else {
        INIT_HIP(hipMemcpyAsync(s->scratch, H0, half, hipMemcpyHostToDevice, s->stream));
        INIT_TRY((convert<float, double>(s->scratch, s->state, 3 * ns, s->stream)));
        INIT_HIP(hipStreamSynchronize(s->stream));
        INIT_HIP(hipMemcpyAsync(s->scratch, E0, half, hipMemcpyHostToDevice, s->stream));
        INIT_TRY((convert<float, double>(s->scratch, (float*)s->state + 3 * ns, 3 * ns, s->stream)));
    }
    INIT_HIP(hipStreamSynchronize(s->stream));
#undef INIT_TRY
#undef INIT_HIP
    *out = s;
    return EIFP_OK;
}

static eifp_status step_impl(eifp_solver* s, double tau, long long nsteps, double* pass_ms) {
    g_err.clear();
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    if (!std::isfinite(tau)) return fail(EIFP_ERR_INVALID_ARG, "tau must be finite");
    if (nsteps < 0) return fail(EIFP_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps == 0) {
        if (pass_ms)
            for (int i = 0; i < 6; ++i) pass_ms[i] = 0.0;
        return EIFP_OK;
    }
    if (pass_ms) {
        const size_t need = (size_t)7 * (size_t)nsteps;
        while (s->events.size() < need) {
            hipEvent_t e;
            HIP_TRY(hipEventCreate(&e));
            s->events.push_back(e);
        }
    }
    for (long long n = 0; n < nsteps; ++n) {
        hipEvent_t* ev = pass_ms ? &s->events[(size_t)7 * n] : nullptr;
        const eifp_status st = passes(s, Z_STEP, s->state, s->state, tau, ev);
        if (st != EIFP_OK) return st;
    }
    s->t += tau * (double)nsteps;
    s->steps += nsteps;
    s->inv_current = true;
    if (pass_ms) {
        HIP_TRY(hipStreamSynchronize(s->stream));
        for (int i = 0; i < 6; ++i) pass_ms[i] = 0.0;
        for (long long n = 0; n < nsteps; ++n) {
            hipEvent_t* ev = &s->events[(size_t)7 * n];
            for (int i = 0; i < 6; ++i) {
                float ms = 0.f;
                HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
                pass_ms[i] += (double)ms;
            }
        }
    }
    return EIFP_OK;
}

eifp_status eifp_step(eifp_solver* s, double tau, long long nsteps) { return step_impl(s, tau, nsteps, nullptr); }

eifp_status eifp_step_timed(eifp_solver* s, double tau, long long nsteps, double* pass_ms) {
    if (!pass_ms) return fail(EIFP_ERR_INVALID_ARG, "pass_ms is NULL");
    return step_impl(s, tau, nsteps, pass_ms);
}

eifp_status eifp_invariants(eifp_solver* s, eifp_invariant_set* out) {
    g_err.clear();
    if (!s || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    if (!s->inv_current) {
        const eifp_status st = passes(s, Z_FORWARD, s->state, s->scratch, 0.0, nullptr);
        if (st != EIFP_OK) return st;
        s->inv_current = true;
    }
    HIP_TRY(hipMemcpyAsync(s->inv_host, s->inv_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    HIP_TRY(hipStreamSynchronize(s->stream));
    const double* v = s->inv_host;
    out->t = s->t;
    out->steps_done = s->steps;
    out->energy = v[0];
    out->helicity = v[1];
    out->momentum[0] = v[2];
    out->momentum[1] = v[3];
    out->momentum[2] = v[4];
    out->div_h_l2 = v[5];
    out->div_e_l2 = v[6];
    for (int i = 0; i < 7; ++i)
        if (!std::isfinite(v[i])) return fail(EIFP_ERR_NONFINITE, "invariant %d is not finite", i);
    return EIFP_OK;
}

eifp_status eifp_fields(eifp_solver* s, double* H, double* E) {
    g_err.clear();
    if (!s || !H || !E) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    const size_t half = (size_t)3 * s->ns * sizeof(double);
    if (s->prec == EIFP_FP64) {
        HIP_TRY(hipMemcpyAsync(H, s->state, half, hipMemcpyDeviceToHost, s->stream));
        HIP_TRY(hipMemcpyAsync(E, (char*)s->state + half, half, hipMemcpyDeviceToHost, s->stream));
    } else {
        for (int part = 0; part < 2; ++part) {
            const eifp_status st = convert<double, float>((const float*)s->state + (size_t)part * 3 * s->ns,
                                                          s->scratch, 3 * s->ns, s->stream);
            if (st != EIFP_OK) return st;
            HIP_TRY(hipMemcpyAsync(part ? E : H, s->scratch, half, hipMemcpyDeviceToHost, s->stream));
            HIP_TRY(hipStreamSynchronize(s->stream));
        }
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

eifp_status eifp_fields_device(eifp_solver* s, void* H, void* E, eifp_precision out_prec) {
    g_err.clear();
    if (!s || !H || !E) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    if (out_prec != EIFP_FP64 && out_prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision");
    const long long n = 3 * s->ns;
    for (int part = 0; part < 2; ++part) {
        void* dst = part ? E : H;
        const char* src = (const char*)s->state + (size_t)part * (size_t)n * s->tsize;
        if (out_prec == s->prec) {
            HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * s->tsize, hipMemcpyDeviceToDevice, s->stream));
        } else {
            const eifp_status st = s->prec == EIFP_FP64 ? convert<float, double>(src, dst, n, s->stream)
                                                        : convert<double, float>(src, dst, n, s->stream);
            if (st != EIFP_OK) return st;
        }
    }
    return EIFP_OK;
}

eifp_status eifp_spectrum(eifp_solver* s, double* out) {
    g_err.clear();
    if (!s || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    const long rows = 6L * s->nz * s->ny;
    const long cs = (long)s->nz * s->ny * s->M;
    int rc;
    if (s->prec == EIFP_FP64) {
        if ((rc = launch_x<double>(false, s->nx, s->state, s->scratch, rows, s->twx, s->stream)))
            return rc_to_status(rc, "x forward");
        if ((rc = launch_y<double>(false, s->ny, s->scratch, s->M, s->nz, s->twy, s->stream)))
            return rc_to_status(rc, "y forward");
        if ((rc = launch_z_fwd_store<double>(s->nz, s->scratch, s->M, s->ny, cs, s->twz, s->stream)))
            return rc_to_status(rc, "z forward");
        HIP_TRY(hipMemcpyAsync(out, s->scratch, s->state_bytes(), hipMemcpyDeviceToHost, s->stream));
    } else {
        if ((rc = launch_x<float>(false, s->nx, s->state, s->scratch, rows, s->twx, s->stream)))
            return rc_to_status(rc, "x forward");
        if ((rc = launch_y<float>(false, s->ny, s->scratch, s->M, s->nz, s->twy, s->stream)))
            return rc_to_status(rc, "y forward");
        if ((rc = launch_z_fwd_store<float>(s->nz, s->scratch, s->M, s->ny, cs, s->twz, s->stream)))
            return rc_to_status(rc, "z forward");
        void* tmp = nullptr;
        const size_t nbytes = (size_t)6 * s->ns * sizeof(double);
        HIP_TRY(hipMalloc(&tmp, nbytes));
        eifp_status st = convert<double, float>(s->scratch, tmp, 6 * s->ns, s->stream);
        if (st == EIFP_OK) {
            hipError_t e = hipMemcpyAsync(out, tmp, nbytes, hipMemcpyDeviceToHost, s->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) st = fail(EIFP_ERR_DEVICE, "spectrum copy failed: %s", hipGetErrorString(e));
        }
        (void)hipFree(tmp);
        if (st != EIFP_OK) return st;
    }
    HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

eifp_status eifp_sync(eifp_solver* s) {
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

void* eifp_stream(eifp_solver* s) { return s ? (void*)s->stream : nullptr; }

long long eifp_device_bytes(eifp_solver* s) { return s ? s->bytes : 0; }

eifp_status eifp_destroy(eifp_solver* s) {
    g_err.clear();
    release(s);
    return EIFP_OK;
}

const char* eifp_status_string(eifp_status st) {
    switch (st) {
        case EIFP_OK: return "ok";
        case EIFP_ERR_INVALID_ARG: return "invalid argument";
        case EIFP_ERR_UNSUPPORTED_SIZE: return "unsupported grid size";
        case EIFP_ERR_OUT_OF_MEMORY: return "out of device memory";
        case EIFP_ERR_DEVICE: return "device error";
        case EIFP_ERR_NONFINITE: return "non-finite value";
        case EIFP_ERR_STATE: return "invalid solver state";
    }
    return "unknown status";
}

const char* eifp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
