// passes_impl.h -- plan and tile selection per axis length, and the launchers.
// Included once per precision (passes_f64.hip, passes_f32.hip).
#pragma once
#include "passes.h"

namespace eifp {

// values per thread for the single-component passes (x, y): radix-16/12 plans
template <int N> struct XYE { static constexpr int E = (N % 3 == 0) ? (N >= 12 ? 12 : N) : (N >= 16 ? 16 : N); };
// values per thread for the fused z pass, which holds six components at once: 4 or 6
// in FP64, 8 or 12 in FP32 (keeps the six pencils in registers without spilling)
#ifndef EIFP_ZE64
#define EIFP_ZE64 4
#endif
#ifndef EIFP_ZE32
#define EIFP_ZE32 8
#endif
template <typename T, int N> struct ZE {
    static constexpr int E2 = sizeof(T) == 8 ? EIFP_ZE64 : EIFP_ZE32;  // for powers of two
    static constexpr int E = sizeof(T) == 8 ? ((N % 3 == 0) ? 6 : (N >= E2 ? E2 : N))
                                            : ((N % 3 == 0) ? (N >= 12 ? 12 : N) : (N >= E2 ? E2 : N));
};

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }

template <typename T, int M> struct XCfg {
    using P = Plan<M, XYE<M>::E>;
    static constexpr int NP = cmax(1, cmin(256 / P::T, (48 * 1024) / ((M + 1) * 2 * (int)sizeof(T))));
};
template <typename T, int N> struct YCfg {
    using P = Plan<N, XYE<N>::E>;
    static constexpr int B = cmax(1, cmin(cmin(64, 256 / P::T), (64 * 1024) / (N * 2 * (int)sizeof(T))));
};
// Row segment (bytes along x) targeted by a z tile; the double-buffered exchange takes
// 4 N B sizeof(T) bytes of LDS.
#ifndef EIFP_ZROW_BYTES
#define EIFP_ZROW_BYTES 128
#endif
template <typename T, int N> struct ZCfg {
    using P = Plan<N, ZE<T, N>::E>;
    // row segments of EIFP_ZROW_BYTES along x, at most 1024 threads and 96 KB of LDS
    static constexpr int B0 = cmin(64, cmax(EIFP_ZROW_BYTES / (2 * (int)sizeof(T)), 256 / P::T));
    static constexpr int B = cmax(1, cmin(cmin(B0, 1024 / P::T), (96 * 1024) / (N * 4 * (int)sizeof(T))));
};

inline int check_launch() { return hipGetLastError() == hipSuccess ? kOk : kLaunchFailed; }

template <typename T, int M>
int run_x(bool inv, const void* src, void* dst, long nrows, const void* twx, hipStream_t st) {
    using C = XCfg<T, M>;
    const dim3 grid((unsigned)((nrows + C::NP - 1) / C::NP));
    const dim3 block(C::P::T * C::NP);
    if (inv)
        hipLaunchKernelGGL((k_x_inv<T, typename C::P, C::NP>), grid, block, 0, st, (const cpx<T>*)src, (cpx<T>*)dst,
                           nrows, (const cpx<T>*)twx);
    else
        hipLaunchKernelGGL((k_x_fwd<T, typename C::P, C::NP>), grid, block, 0, st, (const cpx<T>*)src, (cpx<T>*)dst,
                           nrows, (const cpx<T>*)twx);
    return check_launch();
}

template <typename T, int N>
int run_y(bool inv, void* buf, int M, int nz, const void* twy, hipStream_t st) {
    using C = YCfg<T, N>;
    const dim3 grid((unsigned)((M + C::B - 1) / C::B), (unsigned)nz, 6);
    const dim3 block(C::P::T * C::B);
    if (inv)
        hipLaunchKernelGGL((k_y<T, typename C::P, C::B, true>), grid, block, 0, st, (cpx<T>*)buf, M, nz,
                           (const cpx<T>*)twy);
    else
        hipLaunchKernelGGL((k_y<T, typename C::P, C::B, false>), grid, block, 0, st, (cpx<T>*)buf, M, nz,
                           (const cpx<T>*)twy);
    return check_launch();
}

template <typename T, int N>
int run_z(int mode, void* buf, int M, int ny, long cs, const void* twz, const PropParams& pp, double* partials,
          int want_inv, hipStream_t st) {
    using C = ZCfg<T, N>;
    const dim3 grid((unsigned)((M + C::B - 1) / C::B), (unsigned)ny);
    const dim3 block(C::P::T * C::B);
    if (mode == Z_STEP)
        hipLaunchKernelGGL((k_z<T, typename C::P, C::B, Z_STEP>), grid, block, 0, st, (cpx<T>*)buf, M, ny, cs,
                           (const cpx<T>*)twz, pp, partials, want_inv);
    else
        hipLaunchKernelGGL((k_z<T, typename C::P, C::B, Z_FORWARD>), grid, block, 0, st, (cpx<T>*)buf, M, ny, cs,
                           (const cpx<T>*)twz, pp, partials, want_inv);
    return check_launch();
}

template <typename T, int N>
int count_z(int M, int ny) {
    using C = ZCfg<T, N>;
    return ((M + C::B - 1) / C::B) * ny;
}

template <typename T, int N>
int run_z_store(void* buf, int M, int ny, long cs, const void* twz, hipStream_t st) {
    using C = ZCfg<T, N>;
    const dim3 grid((unsigned)((M + C::B - 1) / C::B), (unsigned)ny, 6);
    const dim3 block(C::P::T * C::B);
    hipLaunchKernelGGL((k_z_fwd_store<T, typename C::P, C::B>), grid, block, 0, st, (cpx<T>*)buf, M, ny, cs,
                       (const cpx<T>*)twz);
    return check_launch();
}

// axis lengths compiled for y and z
#define EIFP_AXIS_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
// half lengths M = Nx/2 compiled for x
#define EIFP_HALF_SIZES(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)

template <typename T>
int launch_x(bool inv, int nx, const void* src, void* dst, long nrows, const void* twx, hipStream_t st) {
    switch (nx / 2) {
#define EIFP_CASE(M) \
    case M:          \
        return run_x<T, M>(inv, src, dst, nrows, twx, st);
        EIFP_HALF_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int launch_y(bool inv, int ny, void* buf, int M, int nz, const void* twy, hipStream_t st) {
    switch (ny) {
#define EIFP_CASE(N) \
    case N:          \
        return run_y<T, N>(inv, buf, M, nz, twy, st);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int launch_z(int mode, int nz, void* buf, int M, int ny, long cs, const void* twz, const PropParams& pp,
             double* partials, int want_inv, hipStream_t st) {
    switch (nz) {
#define EIFP_CASE(N) \
    case N:          \
        return run_z<T, N>(mode, buf, M, ny, cs, twz, pp, partials, want_inv, st);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int z_partial_count(int nz, int M, int ny) {
    switch (nz) {
#define EIFP_CASE(N) \
    case N:          \
        return count_z<T, N>(M, ny);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return -1;
    }
}

template <typename T>
int launch_z_fwd_store(int nz, void* buf, int M, int ny, long cs, const void* twz, hipStream_t st) {
    switch (nz) {
#define EIFP_CASE(N) \
    case N:          \
        return run_z_store<T, N>(buf, M, ny, cs, twz, st);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

#define EIFP_INSTANTIATE(T)                                                                                   \
    template int launch_x<T>(bool, int, const void*, void*, long, const void*, hipStream_t);                  \
    template int launch_y<T>(bool, int, void*, int, int, const void*, hipStream_t);                           \
    template int launch_z<T>(int, int, void*, int, int, long, const void*, const PropParams&, double*, int,    \
                             hipStream_t);                                                                    \
    template int z_partial_count<T>(int, int, int);                                                           \
    template int launch_z_fwd_store<T>(int, void*, int, int, long, const void*, hipStream_t);

}  // namespace eifp
