// solver.hip -- the single-solve object and the C ABI declared in include/eifp.h.
//
// One step (Def. 2.3 / Alg. 2 with t_end = tau) is five kernels on the solver's stream:
//   x forward (R2C split)  ->  z forward  ->  fused y (forward, propagator, invariant
//   partials, inverse)  ->  z inverse (and the finalize of the invariant partials)  ->
//   x inverse (C2R merge)
// The state stays in HBM in the ABI's own layout ([6][nz][ny][nx] reals); a step's
// transforms run in the scratch buffer, and between consecutive steps of one call the
// x inverse and the next x forward are one kernel.
// A solver is a batch of one member: the kernels read its buffers and scalars from a
// four-entry device descriptor array (0: step; 1: forward-only evaluation into the
// scratch buffer; 2: forward transform into the anchor buffer; 3: jump from the anchor).
//
// Jumps: the scheme is the exact flow of the Fourier semi-discretisation for any time
// span (Def. 2.3; Alg. 2 takes t_end in one step), so the state after any number of
// steps can be computed from one stored spectrum (the anchor) by one propagation and
// one inverse transform, with the rounding of one step instead of one per step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

using namespace eifp;

struct eifp_solver {
    Engine en;
    eifp_domain dom{};
    double mu = 1, eps = 1;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    void* state = nullptr;
    void* scratch = nullptr;
    double* partials = nullptr;
    double* inv_dev = nullptr;
    double* inv_host = nullptr;  // pinned
    void* anchor = nullptr;      // anchored spectrum (allocated on first use)
    bool anchor_valid = false;
    double t_anchor = 0.0;
    void* desc_dev = nullptr;    // DescImage[4]
    DescImage desc_host[4]{};
    double desc_tau = 0.0;       // tau held by desc_dev[0]
    double jump_span = 0.0;      // time span held by desc_dev[3]
    bool inv_current = false;    // inv_dev describes the current state
    double t = 0.0;
    long long steps = 0;
    long long bytes = 0;
    std::vector<hipEvent_t> events;
};

namespace {

void release(eifp_solver* s) {
    if (!s) return;
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (void* p : {s->state, s->scratch, s->anchor, (void*)s->partials, (void*)s->inv_dev, s->desc_dev})
        if (p) (void)hipFree(p);
    s->en.release();
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

// Write the descriptors for step size tau and jump span `span`.  The copy is
// synchronous with respect to the host buffer (the stream is drained first), so it
// only happens when tau or the span changes.
eifp_status upload_desc(eifp_solver* s, double tau, double span) {
    const Grid3& g = s->en.g;
    const PropParams p0 = make_params(g.nx, g.ny, g.nz, s->dom, s->mu, s->eps, 0.0);
    // steps transform in the scratch buffer (the x inverse of a step and the x forward
    // of the next then run as one kernel)
    s->desc_host[0] = DescImage{s->state, s->scratch, s->partials, s->inv_dev, nullptr,
                                make_params(g.nx, g.ny, g.nz, s->dom, s->mu, s->eps, tau)};
    s->desc_host[1] = DescImage{s->state, s->scratch, s->partials, s->inv_dev, nullptr, p0};
    s->desc_host[2] = DescImage{s->state, s->anchor, s->partials, s->inv_dev, nullptr, p0};
    s->desc_host[3] = DescImage{s->state, s->state, s->partials, s->inv_dev, s->anchor,
                                make_params(g.nx, g.ny, g.nz, s->dom, s->mu, s->eps, span)};
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    EIFP_HIP_TRY(hipMemcpyAsync(s->desc_dev, s->desc_host, sizeof s->desc_host, hipMemcpyHostToDevice, s->stream));
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    s->desc_tau = tau;
    s->jump_span = span;
    return EIFP_OK;
}

const void* desc_at(const eifp_solver* s, int i) { return (const char*)s->desc_dev + i * sizeof(DescImage); }
const void* step_desc(const eifp_solver* s) { return desc_at(s, 0); }
const void* fwd_desc(const eifp_solver* s) { return desc_at(s, 1); }

// Store the spectrum of the current state as the anchor (time t).
eifp_status make_anchor(eifp_solver* s) {
    eifp_status st;
    if (!s->anchor) {
        if ((st = alloc(&s->anchor, s->en.state_bytes(), &s->bytes))) return st;
        if ((st = upload_desc(s, s->desc_tau, s->jump_span))) return st;
    }
    if ((st = s->en.forward_spectrum(desc_at(s, 2), 1, s->stream))) return st;
    s->anchor_valid = true;
    s->t_anchor = s->t;
    return EIFP_OK;
}

}  // namespace

extern "C" {

eifp_status eifp_init(eifp_solver** out, int nx, int ny, int nz, const eifp_domain* dom, double mu, double eps,
                      eifp_precision prec, const double* H0, const double* E0, void* hip_stream) {
    clear_error();
    if (!out) return fail(EIFP_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!dom || !H0 || !E0) return fail(EIFP_ERR_INVALID_ARG, "NULL domain or field pointer");
    eifp_status st;
    if ((st = validate_shape(nx, ny, nz)) || (st = validate_problem(dom, mu, eps))) return st;
    if (prec != EIFP_FP64 && prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision %d", (int)prec);
    const long long ns = (long long)nx * ny * nz;
    for (long long q = 0; q < 3 * ns; ++q)
        if (!std::isfinite(H0[q]) || !std::isfinite(E0[q]))
            return fail(EIFP_ERR_NONFINITE, "initial field holds NaN/Inf at flat index %lld", q);

    eifp_solver* s = new (std::nothrow) eifp_solver;
    if (!s) return fail(EIFP_ERR_OUT_OF_MEMORY, "host allocation failed");
    s->dom = *dom;
    s->mu = mu;
    s->eps = eps;
#define INIT_TRY(expr)       \
    do {                     \
        st = (expr);         \
        if (st != EIFP_OK) { \
            release(s);      \
            return st;       \
        }                    \
    } while (0)
#define INIT_HIP(expr)                                                                   \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess) {                                                          \
            release(s);                                                                  \
            return fail(EIFP_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
        }                                                                                \
    } while (0)
    if (hip_stream) {
        s->stream = (hipStream_t)hip_stream;
    } else {
        INIT_HIP(hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking));
        s->own_stream = true;
    }
    INIT_TRY(s->en.init(nx, ny, nz, prec, s->stream));
    const size_t sb = s->en.state_bytes();
    INIT_TRY(alloc(&s->state, sb, &s->bytes));
    INIT_TRY(alloc(&s->scratch, sb, &s->bytes));
    INIT_TRY(alloc((void**)&s->partials, s->en.partial_bytes(), &s->bytes));
    INIT_TRY(alloc((void**)&s->inv_dev, INV_XPART * sizeof(double), &s->bytes));
    INIT_TRY(alloc(&s->desc_dev, sizeof s->desc_host, &s->bytes));
    INIT_HIP(hipHostMalloc((void**)&s->inv_host, INV_XPART * sizeof(double), hipHostMallocDefault));
    INIT_TRY(upload_desc(s, 0.0, 0.0));
    // upload: FP64 directly; FP32 through the scratch buffer (3 ns doubles = 6 ns floats)
    const size_t half = (size_t)3 * ns * sizeof(double);
    if (prec == EIFP_FP64) {
        INIT_HIP(hipMemcpyAsync(s->state, H0, half, hipMemcpyHostToDevice, s->stream));
        INIT_HIP(hipMemcpyAsync((char*)s->state + half, E0, half, hipMemcpyHostToDevice, s->stream));
    } else {
        INIT_HIP(hipMemcpyAsync(s->scratch, H0, half, hipMemcpyHostToDevice, s->stream));
        INIT_TRY(convert_f64_to_f32(s->scratch, s->state, 3 * ns, s->stream));
        INIT_HIP(hipStreamSynchronize(s->stream));
        INIT_HIP(hipMemcpyAsync(s->scratch, E0, half, hipMemcpyHostToDevice, s->stream));
        INIT_TRY(convert_f64_to_f32(s->scratch, (float*)s->state + 3 * ns, 3 * ns, s->stream));
    }
    INIT_HIP(hipStreamSynchronize(s->stream));
#undef INIT_TRY
#undef INIT_HIP
    s->bytes += s->en.bytes;
    *out = s;
    return EIFP_OK;
}

static eifp_status step_impl(eifp_solver* s, double tau, long long nsteps, double* pass_ms) {
    clear_error();
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    eifp_status st;
    if ((st = validate_tau(tau))) return st;
    if (nsteps < 0) return fail(EIFP_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps == 0) {
        if (pass_ms)
            for (int i = 0; i < 6; ++i) pass_ms[i] = 0.0;
        return EIFP_OK;
    }
    if (tau != s->desc_tau && (st = upload_desc(s, tau, s->jump_span))) return st;
    s->anchor_valid = false;  // the state no longer follows from the anchor
    if (pass_ms) {
        const size_t need = (size_t)7 * (size_t)nsteps;
        while (s->events.size() < need) {
            hipEvent_t e;
            EIFP_HIP_TRY(hipEventCreate(&e));
            s->events.push_back(e);
        }
    }
    if ((st = s->en.steps(step_desc(s), 1, nsteps, s->stream, pass_ms ? s->events.data() : nullptr, 0, true)))
        return st;
    s->t += tau * (double)nsteps;
    s->steps += nsteps;
    s->inv_current = true;
    if (pass_ms) {
        EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
        for (int i = 0; i < 6; ++i) pass_ms[i] = 0.0;
        for (long long n = 0; n < nsteps; ++n) {
            hipEvent_t* ev = &s->events[(size_t)7 * n];
            for (int i = 0; i < 6; ++i) {
                float ms = 0.f;
                EIFP_HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
                pass_ms[i] += (double)ms;
            }
        }
    }
    return EIFP_OK;
}

eifp_status eifp_step(eifp_solver* s, double tau, long long nsteps) { return step_impl(s, tau, nsteps, nullptr); }

eifp_status eifp_anchor(eifp_solver* s) {
    clear_error();
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    return make_anchor(s);
}

eifp_status eifp_jump(eifp_solver* s, double tau, long long nsteps) {
    clear_error();
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    eifp_status st;
    if ((st = validate_tau(tau))) return st;
    if (nsteps < 0) return fail(EIFP_ERR_INVALID_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return EIFP_OK;
    if (!s->anchor_valid && (st = make_anchor(s))) return st;
    const double t_new = s->t + tau * (double)nsteps;
    const double span = t_new - s->t_anchor;
    if (!std::isfinite(span)) return fail(EIFP_ERR_INVALID_ARG, "time span is not finite");
    if (span != s->jump_span && (st = upload_desc(s, s->desc_tau, span))) return st;
    if ((st = s->en.jump(desc_at(s, 3), 1, s->stream))) return st;
    s->t = t_new;
    s->steps += nsteps;
    s->inv_current = true;
    return EIFP_OK;
}

eifp_status eifp_step_timed(eifp_solver* s, double tau, long long nsteps, double* pass_ms) {
    if (!pass_ms) return fail(EIFP_ERR_INVALID_ARG, "pass_ms is NULL");
    return step_impl(s, tau, nsteps, pass_ms);
}

eifp_status eifp_invariants(eifp_solver* s, eifp_invariant_set* out) {
    clear_error();
    if (!s || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    if (!s->inv_current) {
        const eifp_status st = s->en.passes(Z_FORWARD, fwd_desc(s), 1, s->stream, nullptr);
        if (st != EIFP_OK) return st;
        s->inv_current = true;
    }
    EIFP_HIP_TRY(hipMemcpyAsync(s->inv_host, s->inv_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
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

eifp_status eifp_invariants_ext(eifp_solver* s, eifp_invariant_ext_set* out) {
    clear_error();
    if (!s || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    eifp_status st = s->en.passes(Z_FORWARD_EXT, fwd_desc(s), 1, s->stream, nullptr);
    if (st != EIFP_OK) return st;
    s->inv_current = true;  // the basic record is rewritten for the same state
    EIFP_HIP_TRY(hipMemcpyAsync(s->inv_host, s->inv_dev, INV_XPART * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    const double* v = s->inv_host;
    out->t = s->t;
    out->steps_done = s->steps;
    out->e2 = v[INV_E2];
    for (int k = 0; k < 3; ++k) {
        out->e3[k] = v[INV_E3X + k];
        out->e4[k] = v[INV_E4X + k];
    }
    out->h2 = v[INV_H2];
    out->scale_helicity = v[INV_SH1];
    for (int k = 0; k < 3; ++k) out->scale_momentum[k] = std::sqrt(v[INV_HH]) * std::sqrt(v[INV_BEX + k]);
    out->scale_div_h = s->mu * std::sqrt(v[INV_B2H]);
    out->scale_div_e = s->eps * std::sqrt(v[INV_B2E]);
    for (int q = INV_NPART; q < INV_XPART; ++q)
        if (!std::isfinite(v[q])) return fail(EIFP_ERR_NONFINITE, "extended invariant %d is not finite", q);
    return EIFP_OK;
}

eifp_status eifp_fields(eifp_solver* s, double* H, double* E) {
    clear_error();
    if (!s || !H || !E) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    const long long ns = s->en.ns;
    const size_t half = (size_t)3 * ns * sizeof(double);
    if (s->en.prec == EIFP_FP64) {
        EIFP_HIP_TRY(hipMemcpyAsync(H, s->state, half, hipMemcpyDeviceToHost, s->stream));
        EIFP_HIP_TRY(hipMemcpyAsync(E, (char*)s->state + half, half, hipMemcpyDeviceToHost, s->stream));
    } else {
        for (int part = 0; part < 2; ++part) {
            const eifp_status st =
                convert_f32_to_f64((const float*)s->state + (size_t)part * 3 * ns, s->scratch, 3 * ns, s->stream);
            if (st != EIFP_OK) return st;
            EIFP_HIP_TRY(hipMemcpyAsync(part ? E : H, s->scratch, half, hipMemcpyDeviceToHost, s->stream));
            EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
        }
    }
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

eifp_status eifp_fields_device(eifp_solver* s, void* H, void* E, eifp_precision out_prec) {
    clear_error();
    if (!s || !H || !E) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    if (out_prec != EIFP_FP64 && out_prec != EIFP_FP32) return fail(EIFP_ERR_INVALID_ARG, "unknown precision");
    const long long n = 3 * s->en.ns;
    const size_t ts = s->en.tsize;
    for (int part = 0; part < 2; ++part) {
        void* dst = part ? E : H;
        const char* src = (const char*)s->state + (size_t)part * (size_t)n * ts;
        if (out_prec == s->en.prec) {
            EIFP_HIP_TRY(hipMemcpyAsync(dst, src, (size_t)n * ts, hipMemcpyDeviceToDevice, s->stream));
        } else {
            const eifp_status st = s->en.prec == EIFP_FP64 ? convert_f64_to_f32(src, dst, n, s->stream)
                                                           : convert_f32_to_f64(src, dst, n, s->stream);
            if (st != EIFP_OK) return st;
        }
    }
    return EIFP_OK;
}

eifp_status eifp_spectrum(eifp_solver* s, double* out) {
    clear_error();
    if (!s || !out) return fail(EIFP_ERR_INVALID_ARG, "NULL argument");
    eifp_status st = s->en.forward_spectrum(fwd_desc(s), 1, s->stream);
    if (st != EIFP_OK) return st;
    const long long ns = s->en.ns;
    if (s->en.prec == EIFP_FP64) {
        EIFP_HIP_TRY(hipMemcpyAsync(out, s->scratch, s->en.state_bytes(), hipMemcpyDeviceToHost, s->stream));
    } else {
        void* tmp = nullptr;
        const size_t nbytes = (size_t)6 * ns * sizeof(double);
        EIFP_HIP_TRY(hipMalloc(&tmp, nbytes));
        st = convert_f32_to_f64(s->scratch, tmp, 6 * ns, s->stream);
        if (st == EIFP_OK) {
            hipError_t e = hipMemcpyAsync(out, tmp, nbytes, hipMemcpyDeviceToHost, s->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
            if (e != hipSuccess) st = fail(EIFP_ERR_DEVICE, "spectrum copy failed: %s", hipGetErrorString(e));
        }
        (void)hipFree(tmp);
        if (st != EIFP_OK) return st;
    }
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

eifp_status eifp_sync(eifp_solver* s) {
    if (!s) return fail(EIFP_ERR_INVALID_ARG, "solver is NULL");
    EIFP_HIP_TRY(hipStreamSynchronize(s->stream));
    return EIFP_OK;
}

void* eifp_stream(eifp_solver* s) { return s ? (void*)s->stream : nullptr; }

long long eifp_device_bytes(eifp_solver* s) { return s ? s->bytes : 0; }

eifp_status eifp_destroy(eifp_solver* s) {
    clear_error();
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
        case EIFP_ERR_CANCELLED: return "request cancelled";
    }
    return "unknown status";
}

const char* eifp_last_error(void) { return last_error(); }

}  // extern "C"
