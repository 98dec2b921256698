// passes_impl.h -- plan and tile selection per axis length, and the launchers.
// Included once per precision (passes_f64.hip, passes_f32.hip).
#pragma once
#include "passes.h"
#include "small_plane.h"

namespace eifp {

// values per thread for the single-component passes (x, y, z): radix-16/12 plans
template <int N> struct XYE { static constexpr int E = (N % 3 == 0) ? (N >= 12 ? 12 : N) : (N >= 16 ? 16 : N); };
// values per thread for the fused pass, which holds six components at once: 8 in FP64,
// with one wave per SIMD and the accumulation registers as the overflow of the six
// pencils; 8 in FP32 at two waves per SIMD; lengths with a factor 3 below (their
// split form holds three components per thread)
#ifndef EIFP_ZE64
#define EIFP_ZE64 8
#endif
#ifndef EIFP_ZE32
#define EIFP_ZE32 8
#endif
template <typename T, int N> struct ZE {
    static constexpr int E2 = sizeof(T) == 8 ? EIFP_ZE64 : EIFP_ZE32;  // for powers of two
    // lengths with a factor 3: 6 per thread in FP64, 12 in FP32 (fewer stages)
    static constexpr int E3 = sizeof(T) == 8 ? 6 : 12;
    static constexpr int E = (N % 3 == 0) ? (N >= E3 ? E3 : N) : (N >= E2 ? E2 : N);
};

constexpr int cmin(int a, int b) { return a < b ? a : b; }
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int pow2floor(int a) {  // largest power of two <= a (a >= 1)
    int p = 1;
    while (2 * p <= a) p *= 2;
    return p;
}

// LDS budget of the x pass's row buffers per workgroup (rows of 2.3 KB in FP64 at
// length 128: 21 rows, three workgroups per CU)
#ifndef EIFP_XLDS_KB
#define EIFP_XLDS_KB 48
#endif
template <typename T, int M> struct XCfg {
    using P = Plan<M, XYE<M>::E>;
    static constexpr int NP = cmax(1, cmin(256 / P::T, (EIFP_XLDS_KB * 1024) / (rows_pitch<T>(M) * 2 * (int)sizeof(T))));
};

// Row segment (bytes along x) of a tile of the single-component strided pass.
#ifndef EIFP_CROW_BYTES
#define EIFP_CROW_BYTES 256
#endif
// LDS budget of the strided pass's exchange per workgroup
#ifndef EIFP_CLDS_KB
#define EIFP_CLDS_KB 80
#endif
template <typename T, int N> struct CCfg {
    using P = Plan<N, XYE<N>::E>;
    static constexpr int B0 = cmin(64, cmax(EIFP_CROW_BYTES / (2 * (int)sizeof(T)), 256 / P::T));
    // at most 1024 threads and 80 KB of LDS ([pos][col] pitch B + pad, two planes), a
    // power of two so that tiles stay aligned to the row segments
    static constexpr int B = pow2floor(
        cmax(1, cmin(cmin(B0, 1024 / P::T),
                     (EIFP_CLDS_KB * 1024) / (skew_rows<N, c2c_skew<P>()>() * 2 * (int)sizeof(T)) - EIFP_LDS_PAD)));
};

// Row segment targeted by a tile of the fused pass; its double-buffered exchange takes
// 4 N (B + pad) sizeof(T) bytes of LDS.
// Tiles of the fused pass are narrow (64-byte row segments; 128-thread workgroups at
// the least) so that two or more workgroups share a CU and overlap their load, compute
// and store phases; the tiles are numbered XCD by XCD (xcd_tiles) so that the two
// halves of a 128-byte line are read by the same L2.
#ifndef EIFP_ZROW_BYTES
#define EIFP_ZROW_BYTES 64
#endif
#ifndef EIFP_ZMIN_THREADS
#define EIFP_ZMIN_THREADS 128
#endif
// LDS budget of the fused pass's exchange buffers per workgroup
#ifndef EIFP_ZLDS_KB
#define EIFP_ZLDS_KB 96
#endif
// At most 256 threads per fused workgroup, so that two share a CU (FP32 length 512 would
// otherwise take one 512-thread workgroup per CU; with 32-byte rows its pass is 20%
// faster at 512^3).
#ifndef EIFP_ZMAX_THREADS
#define EIFP_ZMAX_THREADS 256
#endif
template <typename T, int N> struct ZCfg {
    using P = Plan<N, ZE<T, N>::E>;
    static constexpr int B0 = cmin(cmax(1, EIFP_ZMAX_THREADS / P::T),
                                   cmin(64, cmax(EIFP_ZROW_BYTES / (2 * (int)sizeof(T)), EIFP_ZMIN_THREADS / P::T)));
    static constexpr int B = pow2floor(
        cmax(1, cmin(cmin(B0, 1024 / P::T), (EIFP_ZLDS_KB * 1024) / (skew_rows<N, zskew<P>()>() * 4 * (int)sizeof(T) * ZLockstep<T, N>::value) -
                         EIFP_ZPAD)));
};

// The split fused pass (two thread groups per tile, one per field) holds half the
// registers per thread; each group must be whole waves, so narrow tiles of short
// pencils are widened to 64 / T columns.  Its exchange buffers take 8 N (B + pad)
// sizeof(T) bytes of LDS, kept within 120 KB.
// 0: never; 1: lengths with a factor 3; 2: every length
#ifndef EIFP_FUSED_SPLIT
#define EIFP_FUSED_SPLIT 1
#endif
// values per thread in the split form for lengths with a factor 3: 12 in FP32, and in
// FP64 from length 192 (a thread holds three components, so FP64 affords the plan with
// fewer stages: 192 = 12 4 4 instead of 6 2 2 2 2 2, 4% off the 192^3 pass at one wave
// per SIMD); shorter FP64 lengths keep 6 at two waves, since their few tiles would not
// fill the device at one wave
#ifndef EIFP_ZSE3_64
#define EIFP_ZSE3_64 12
#endif
#ifndef EIFP_ZSE3_64_FROM
#define EIFP_ZSE3_64_FROM 192
#endif
template <typename T, int N> struct ZES {
    static constexpr int E3 = sizeof(T) == 8 ? (N >= EIFP_ZSE3_64_FROM ? EIFP_ZSE3_64 : 6) : 12;
    static constexpr int E = (N % 3 == 0) ? (N >= E3 ? E3 : N) : ZE<T, N>::E;
};
template <typename T, int N> struct ZCfgS {
    using P = Plan<N, ZES<T, N>::E>;
    static constexpr int Bmin = cmax(1, 64 / P::T);
    static constexpr int B0 = cmax(Bmin, cmin(64, EIFP_ZROW_BYTES / (2 * (int)sizeof(T))));
    static constexpr int Bl = pow2floor(cmax(1, (120 * 1024) / (8 * skew_rows<N, zskew<P>()>() * (int)sizeof(T)) - EIFP_ZPAD));
    static constexpr int B = cmin(cmin(B0, Bl), 512 / P::T);
    static constexpr bool ok =
        (EIFP_FUSED_SPLIT == 2 || (EIFP_FUSED_SPLIT == 1 && N % 3 == 0)) && B >= Bmin && P::E % 2 == 0;
};

inline int check_launch() { return hipGetLastError() == hipSuccess ? kOk : kLaunchFailed; }

// axis strides (complex elements): pencil stride, outer stride, outer count
struct AxisGeom {
    long pstride, ostride;
    int n_outer;
};
inline AxisGeom axis_geom(int axis, const Grid3& g) {
    if (axis == AXIS_Y) return {(long)g.M, (long)g.ny * g.M, g.nz};
    return {(long)g.ny * g.M, (long)g.M, g.ny};
}

// Non-temporal stores of the z passes for states above half of the 256 MB last-level
// cache (a state that small stays cached from pass to pass).
#ifndef EIFP_NT_STATE_MB
#define EIFP_NT_STATE_MB 128
#endif
inline bool nt_state(const Grid3& g, size_t tsize) {
    return 6.0 * g.nx * g.ny * g.nz * (double)tsize > EIFP_NT_STATE_MB * 1048576.0;
}

template <typename T, int M>
int run_x(int kind, const Grid3& g, const void* md, int nm, const void* twx, hipStream_t st, int fin_nparts) {
    using C = XCfg<T, M>;
    const long nrows = 6L * g.nz * g.ny;
    const unsigned nblk = (unsigned)((nrows + C::NP - 1) / C::NP);
    const dim3 grid(nblk, (unsigned)nm);
    const dim3 block(C::P::T * C::NP);
    const MemberDesc<T>* d = (const MemberDesc<T>*)md;
    if (fin_nparts > 0) {  // one more workgroup per member: the finalize
        if (kind == X_INV)
            hipLaunchKernelGGL((k_x_inv_fin<T, typename C::P, C::NP>), dim3(nblk + 1, nm), block, 0, st, d, nrows,
                               (const cpx<T>*)twx, fin_nparts);
        else if (kind == X_INVFWD)
            hipLaunchKernelGGL((k_x_invfwd_fin<T, typename C::P, C::NP>), dim3(nblk + 1, nm), block, 0, st, d,
                               nrows, (const cpx<T>*)twx, fin_nparts);
        else
            return kUnsupported;
        return check_launch();
    }
    if (kind == X_INV)
        hipLaunchKernelGGL((k_x_inv<T, typename C::P, C::NP>), grid, block, 0, st, d, nrows, (const cpx<T>*)twx);
    else if (kind == X_INVFWD)
        hipLaunchKernelGGL((k_x_invfwd<T, typename C::P, C::NP>), grid, block, 0, st, d, nrows, (const cpx<T>*)twx);
    else
        hipLaunchKernelGGL((k_x_fwd<T, typename C::P, C::NP>), grid, block, 0, st, d, nrows, (const cpx<T>*)twx);
    return check_launch();
}

template <typename T, int N>
int run_c2c(bool inv, int axis, const Grid3& g, const void* md, int nm, const void* tw, hipStream_t st,
            int fin_nparts, int comp_desc) {
    using C = CCfg<T, N>;
    const AxisGeom a = axis_geom(axis, g);
    const unsigned ntx = (unsigned)((g.M + C::B - 1) / C::B) + (fin_nparts > 0 ? 1u : 0u);
    const dim3 grid(ntx, (unsigned)a.n_outer, (unsigned)(6 * nm));
    const dim3 block(C::P::T * C::B);
    const MemberDesc<T>* d = (const MemberDesc<T>*)md;
    // large states: non-temporal stores (see kStoreNT)
    const bool nt = nt_state(g, sizeof(T));
    if (inv && nt)
        hipLaunchKernelGGL((k_c2c<T, typename C::P, C::B, true, kStoreNT>), grid, block, 0, st, d, g.M, a.pstride,
                           a.ostride, g.cs(), (const cpx<T>*)tw, fin_nparts, 0);
    else if (inv)
        hipLaunchKernelGGL((k_c2c<T, typename C::P, C::B, true>), grid, block, 0, st, d, g.M, a.pstride, a.ostride,
                           g.cs(), (const cpx<T>*)tw, fin_nparts, 0);
    else if (nt)
        hipLaunchKernelGGL((k_c2c<T, typename C::P, C::B, false, kStoreNT>), grid, block, 0, st, d, g.M, a.pstride,
                           a.ostride, g.cs(), (const cpx<T>*)tw, fin_nparts, comp_desc);
    else
        hipLaunchKernelGGL((k_c2c<T, typename C::P, C::B, false>), grid, block, 0, st, d, g.M, a.pstride, a.ostride,
                           g.cs(), (const cpx<T>*)tw, fin_nparts, comp_desc);
    return check_launch();
}

// Workgroups of the persistent fused pass (one partial record each; one per tile when
// the precision's pass is not persistent): as many as the device holds at once (CUs times the step kernel's resident workgroups per CU), a
// multiple of 8 when there are at least 8, at most one per tile.  The residency is
// queried once per process; without a device (host-only use) every tile gets its own
// workgroup.  Every mode uses the step kernel's count, so the partial buffers and the
// finalize agree on it.
// The fused pass's configuration for length N: the split form (k_fused_split) or the
// six-components-per-thread form (k_fused), its tile width, threads and persistence.
template <typename T, int N, int AXIS> struct FusedSel {
    static constexpr bool split = ZCfgS<T, N>::ok;
    static constexpr int B = split ? ZCfgS<T, N>::B : ZCfg<T, N>::B;
    static constexpr int threads = split ? 2 * ZCfgS<T, N>::P::T * ZCfgS<T, N>::B : ZCfg<T, N>::P::T * ZCfg<T, N>::B;
    static constexpr bool persist =
        split ? ZPersistS<T, typename ZCfgS<T, N>::P>::value : ZPersist<T>::value;
    static const void* step_kernel() {
        if constexpr (split)
            return (const void*)k_fused_split<T, typename ZCfgS<T, N>::P, ZCfgS<T, N>::B, Z_STEP, AXIS>;
        else
            return (const void*)k_fused<T, typename ZCfg<T, N>::P, ZCfg<T, N>::B, Z_STEP, AXIS>;
    }
};

template <typename T, int N, int AXIS>
int fused_workgroups(const Grid3& g) {
    using S = FusedSel<T, N, AXIS>;
    const int ntiles = ((g.M + S::B - 1) / S::B) * axis_geom(AXIS, g).n_outer;
    if (!S::persist) return ntiles;
    static const int resident = [] {
        int dev = 0, cus = 0, nb = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, S::step_kernel(), S::threads, 0) != hipSuccess ||
            cus <= 0 || nb <= 0) {
            (void)hipGetLastError();  // leave no error behind for the next launch check
            return 0;
        }
        return cus * nb;
    }();
    if (resident <= 0 || resident >= ntiles) return ntiles;
    return resident >= 8 ? resident & ~7 : resident;
}

template <typename T, int N, int MODE, int AXIS>
void run_fused_k(const Grid3& g, const void* md, int nm, const void* tw, int want_inv, hipStream_t st) {
    const AxisGeom a = axis_geom(AXIS, g);
    if constexpr (ZCfgS<T, N>::ok) {
        using C = ZCfgS<T, N>;
        const int ntx = (g.M + C::B - 1) / C::B;
        const dim3 grid((unsigned)fused_workgroups<T, N, AXIS>(g), 1u, (unsigned)nm);
        const dim3 block(2 * C::P::T * C::B);
        hipLaunchKernelGGL((k_fused_split<T, typename C::P, C::B, MODE, AXIS>), grid, block, 0, st,
                           (const MemberDesc<T>*)md, g.M, a.n_outer, ntx, a.pstride, a.ostride, g.cs(),
                           (const cpx<T>*)tw, want_inv);
    } else {
        using C = ZCfg<T, N>;
        const int ntx = (g.M + C::B - 1) / C::B;
        const dim3 grid((unsigned)fused_workgroups<T, N, AXIS>(g), 1u, (unsigned)nm);
        const dim3 block(C::P::T * C::B);
        hipLaunchKernelGGL((k_fused<T, typename C::P, C::B, MODE, AXIS>), grid, block, 0, st,
                           (const MemberDesc<T>*)md, g.M, a.n_outer, ntx, a.pstride, a.ostride, g.cs(),
                           (const cpx<T>*)tw, want_inv);
    }
}

template <typename T, int N>
int run_fused(int mode, int axis, const Grid3& g, const void* md, int nm, const void* tw, int want_inv,
              hipStream_t st) {
    // only the y-fused form is compiled (the step's pass order); the kernel template
    // also covers z-fused pencils
    if (axis != AXIS_Y) return kUnsupported;
    if (mode == Z_STEP) run_fused_k<T, N, Z_STEP, AXIS_Y>(g, md, nm, tw, want_inv, st);
    else if (mode == Z_FORWARD) run_fused_k<T, N, Z_FORWARD, AXIS_Y>(g, md, nm, tw, want_inv, st);
    else if (mode == Z_JUMP) run_fused_k<T, N, Z_JUMP, AXIS_Y>(g, md, nm, tw, want_inv, st);
    else if (mode == Z_FORWARD_EXT) run_fused_k<T, N, Z_FORWARD_EXT, AXIS_Y>(g, md, nm, tw, want_inv, st);
    else return kUnsupported;
    return check_launch();
}

template <typename T, int N>
int count_fused(int axis, const Grid3& g) {
    return axis == AXIS_Y ? fused_workgroups<T, N, AXIS_Y>(g) : -1;
}

// axis lengths compiled for y and z (a build may list fewer, e.g. to time one size)
#ifndef EIFP_AXIS_SIZES
#define EIFP_AXIS_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)
#endif
// half lengths M = Nx/2 compiled for x
#ifndef EIFP_HALF_SIZES
#define EIFP_HALF_SIZES(X) X(2) X(3) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256)
#endif

inline int axis_len(int axis, const Grid3& g) { return axis == AXIS_Y ? g.ny : g.nz; }

template <typename T>
int launch_x(int kind, const Grid3& g, const void* md, int nm, const void* twx, hipStream_t st, int fin_nparts) {
    switch (g.M) {
#define EIFP_CASE(MM) \
    case MM:          \
        return run_x<T, MM>(kind, g, md, nm, twx, st, fin_nparts);
        EIFP_HALF_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int launch_c2c(bool inv, int axis, const Grid3& g, const void* md, int nm, const void* tw, hipStream_t st,
               int fin_nparts, int comp_desc) {
    switch (axis_len(axis, g)) {
#define EIFP_CASE(N) \
    case N:          \
        return run_c2c<T, N>(inv, axis, g, md, nm, tw, st, fin_nparts, comp_desc);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int launch_fused(int mode, int axis, const Grid3& g, const void* md, int nm, const void* tw, int want_inv,
                 hipStream_t st) {
    switch (axis_len(axis, g)) {
#define EIFP_CASE(N) \
    case N:          \
        return run_fused<T, N>(mode, axis, g, md, nm, tw, want_inv, st);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int fused_partial_count(int axis, const Grid3& g) {
    switch (axis_len(axis, g)) {
#define EIFP_CASE(N) \
    case N:          \
        return count_fused<T, N>(axis, g);
        EIFP_AXIS_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return -1;
    }
}

// plane pass: pencil lengths with a single-thread plan, and a plane of the six
// components within the LDS budget (below two workgroups' worth at FP64 32 x 32)
#ifndef EIFP_PLANE_SIZES
#define EIFP_PLANE_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32)
#endif
// 0 switches the plane pass off (every grid takes the strided passes)
#ifndef EIFP_PLANE
#define EIFP_PLANE 1
#endif
inline bool plane_len(int n) {
    switch (n) {
#define EIFP_CASE(N) \
    case N:          \
        return true;
        EIFP_PLANE_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return false;
    }
}
// Plane pass only where it is the faster path: planes of up to 576 points, where a
// step is dominated by the per-launch cost (us per FP64 step, plane / strided: 8^3 9.7 /
// 21.6, 16^3 13.7 / 25.2, 256 x 16^2 22.5 / 33.6, 32 x 16 x 32 23.0 / 29.0, 24^3 23.9 /
// 24.6).  A 32 x 32 plane is 13% slower than the strided passes: its workgroup takes a
// whole CU and only M of them run.
#ifndef EIFP_PLANE_MAX_POINTS
#define EIFP_PLANE_MAX_POINTS 576
#endif
template <typename T>
bool plane_ok(const Grid3& g) {
    return EIFP_PLANE && plane_len(g.ny) && plane_len(g.nz) && g.ny * g.nz <= EIFP_PLANE_MAX_POINTS &&
           6L * g.ny * g.nz * (long)sizeof(cpx<T>) <= 96L * 1024;
}
template <typename T, int NY, int NZ>
int run_plane(const Grid3& g, const void* md, int nm, const void* twy, const void* twz, int want_inv, hipStream_t st) {
    hipLaunchKernelGGL((k_yz_plane<T, NY, NZ>), dim3((unsigned)g.M, (unsigned)nm), dim3(kPlaneThreads), 0, st,
                       (const MemberDesc<T>*)md, g.M, g.cs(), (const cpx<T>*)twy, (const cpx<T>*)twz, want_inv);
    return check_launch();
}
template <typename T, int NY>
int run_plane_z(const Grid3& g, const void* md, int nm, const void* twy, const void* twz, int want_inv, hipStream_t st) {
    switch (g.nz) {
#define EIFP_CASE(N) \
    case N:          \
        return run_plane<T, NY, N>(g, md, nm, twy, twz, want_inv, st);
        EIFP_PLANE_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}
template <typename T>
int launch_plane(const Grid3& g, const void* md, int nm, const void* twy, const void* twz, int want_inv,
                 hipStream_t st) {
    if (!plane_ok<T>(g)) return kUnsupported;
    switch (g.ny) {
#define EIFP_CASE(N) \
    case N:          \
        return run_plane_z<T, N>(g, md, nm, twy, twz, want_inv, st);
        EIFP_PLANE_SIZES(EIFP_CASE)
#undef EIFP_CASE
        default:
            return kUnsupported;
    }
}

template <typename T>
int launch_finalize(const void* md, int nm, int nparts, hipStream_t st, bool extended) {
    if (extended)
        hipLaunchKernelGGL((k_finalize<T, INV_XPART>), dim3(nm), dim3(1024), 0, st, (const MemberDesc<T>*)md, nparts);
    else
        hipLaunchKernelGGL((k_finalize<T, INV_NPART>), dim3(nm), dim3(1024), 0, st, (const MemberDesc<T>*)md, nparts);
    return check_launch();
}

// The strided single-component passes are instantiated in translation units of their own
// (passes_c2c_f64.hip, passes_c2c_f32.hip), which the build compiles with a scheduling
// strategy that measured faster for them alone.
#define EIFP_INSTANTIATE_C2C(T) \
    template int launch_c2c<T>(bool, int, const Grid3&, const void*, int, const void*, hipStream_t, int, int);
#define EIFP_INSTANTIATE(T)                                                                                   \
    template int launch_x<T>(int, const Grid3&, const void*, int, const void*, hipStream_t, int);             \
    template bool plane_ok<T>(const Grid3&);                                                                 \
    template int launch_plane<T>(const Grid3&, const void*, int, const void*, const void*, int, hipStream_t); \
    template int launch_fused<T>(int, int, const Grid3&, const void*, int, const void*, int, hipStream_t);    \
    template int fused_partial_count<T>(int, const Grid3&);                                                   \
    template int launch_finalize<T>(const void*, int, int, hipStream_t, bool);

}  // namespace eifp
