// small_plane.h -- the y and z work of one step for grids whose (y, z) plane of all six
// components fits in LDS: one workgroup per packed x column.
//
// After the x pass, a column kx of the packed half spectrum holds, for each component,
// the Ny x Nz plane of coefficients (kx, y, z).  The forward transforms along z and y,
// the mode-wise propagator (Prop. 2.1/2.2, Alg. 2 step 4) with the invariant partial
// sums, and the inverse transforms along y and z touch only that plane, so one
// workgroup can take the whole plane into LDS and run them there, with one launch in
// place of the three (z forward, fused y, z inverse) the strided passes need.  For small
// grids each launch costs several microseconds of dispatch and completion whatever its
// size, so this halves the kernels of a step.  Each pencil of the plane (length <= 32)
// is transformed by one thread in its registers, with the same plans' butterflies and
// the same FP64-formed twiddle tables as the strided passes.
#pragma once
#include "kernels.h"

namespace eifp {

// Exchanges of a single-thread plan (T = 1): the "positions" are the thread's own values,
// so the exchange is a renaming of registers (every index is a compile-time constant).
template <typename T, int N>
struct RegExchange {
    cpx<T> a[N];
    __device__ __forceinline__ void st(int pos, cpx<T> v) { a[pos] = v; }
    __device__ __forceinline__ cpx<T> ld(int pos) const { return a[pos]; }
    __device__ __forceinline__ void sync() {}
    __device__ __forceinline__ void after_load() {}
};

// single-thread plans for the plane's pencil lengths (4 ... 16 are the strided passes'
// one-radix plans)
template <> struct Plan<24, 24> : PlanDef<24, 24, 12, 2> {};
template <> struct Plan<32, 32> : PlanDef<32, 32, 16, 2> {};
template <int N> struct PencilPlan { using P = Plan<N, N>; };

// Transform the pencil base[m * stride], m < N, in place: read in the plan's first-stage
// order, write in its last-stage order (natural order in and out).
template <typename T, int N, bool INV>
__device__ __forceinline__ void plane_pencil(cpx<T>* base, int stride, const cpx<T>* tw) {
    using P = typename PencilPlan<N>::P;
    cpx<T> v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = base[m_first<P>(i) * stride];
    RegExchange<T, N> x;
    fft_pencil<P, INV, 1>(v, 0, x, tw);
#pragma unroll
    for (int i = 0; i < N; ++i) base[m_last<P>(i) * stride] = v[i];
}

constexpr int kPlaneThreads = 256;

// Grid: (M columns, members).  Column kx of component c is the plane of elements
// work[c cs + (z Ny + y) M + kx]; it is held in LDS as [c][z][y] with a row pitch of
// Ny + 1 elements, so that the lanes of a wave walking y-pencils (kz apart) spread over
// the banks.  twy, twz: the engine's tables for Ny and Nz (entries, then the FP32
// remainders).  One partial record of the basic invariants per workgroup, at index kx of
// the member's partials (summed by the x kernel that follows, k_x_inv_fin or
// k_x_invfwd_fin).
template <typename T, int NY, int NZ>
__global__ void __launch_bounds__(kPlaneThreads)
k_yz_plane(const MemberDesc<T>* __restrict__ md, int M, long cs, const cpx<T>* __restrict__ twy,
           const cpx<T>* __restrict__ twz, int want_inv) {
    constexpr int NT = kPlaneThreads, NYP = NY + 1, PL = NY * NZ, PLP = NZ * NYP;
    __shared__ cpx<T> s_p[6 * PLP];
    __shared__ cpx<T> s_ty[NY * TwParts<T>::value];
    __shared__ cpx<T> s_tz[NZ * TwParts<T>::value];
    __shared__ double s_red[(NT / 64) * INV_NPART];
    const MemberDesc<T>& mem = md[blockIdx.y];
    const PropParams pp = mem.pp;
    cpx<T>* buf = mem.work;
    const int kx = (int)blockIdx.x;
    for (int i = threadIdx.x; i < NY * TwParts<T>::value; i += NT) s_ty[i] = twy[i];
    for (int i = threadIdx.x; i < NZ * TwParts<T>::value; i += NT) s_tz[i] = twz[i];
    for (int i = threadIdx.x; i < 6 * PL; i += NT) {
        const int c = i / PL, r = i - c * PL, z = r / NY, y = r - z * NY;  // r = z Ny + y
        s_p[c * PLP + z * NYP + y] = buf[c * cs + (long)r * M + kx];
    }
    __syncthreads();
    // forward along z (pencils (c, y), stride Ny + 1), then along y (pencils (c, kz))
    for (int p = threadIdx.x; p < 6 * NY; p += NT)
        plane_pencil<T, NZ, false>(s_p + (p / NY) * PLP + p % NY, NYP, s_tz);
    __syncthreads();
    for (int p = threadIdx.x; p < 6 * NZ; p += NT)
        plane_pencil<T, NY, false>(s_p + (p / NZ) * PLP + (p % NZ) * NYP, 1, s_ty);
    __syncthreads();
    // modes (ky, kz): propagate, and sum the invariants of the new state, as the fused
    // pass does (packed column 0 holds kx = 0 and Nx/2, both with Omega_x = 0, weight 1)
    const double bx = kx == 0 ? 0.0 : pp.nu[0] * (double)kx;
    const double w = kx == 0 ? 1.0 : 2.0;
    double acc[INV_NPART];
#pragma unroll
    for (int q = 0; q < INV_NPART; ++q) acc[q] = 0.0;
    for (int m = threadIdx.x; m < PL; m += NT) {
        const int kz = m / NY, ky = m - kz * NY, a = kz * NYP + ky;
        const double by = omega(ky, NY, pp.nu[1]), bz = omega(kz, NZ, pp.nu[2]);
        cpx<T> h[3] = {s_p[a], s_p[PLP + a], s_p[2 * PLP + a]};
        cpx<T> e[3] = {s_p[3 * PLP + a], s_p[4 * PLP + a], s_p[5 * PLP + a]};
        propagate_mode(h, e, bx, by, bz, pp);
        if (want_inv) accumulate_invariants<INV_NPART>(acc, w, bx, by, bz, h, e, pp);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            s_p[q * PLP + a] = h[q];
            s_p[(3 + q) * PLP + a] = e[q];
        }
    }
    __syncthreads();
    // inverse along y, then along z
    for (int p = threadIdx.x; p < 6 * NZ; p += NT)
        plane_pencil<T, NY, true>(s_p + (p / NZ) * PLP + (p % NZ) * NYP, 1, s_ty);
    __syncthreads();
    for (int p = threadIdx.x; p < 6 * NY; p += NT)
        plane_pencil<T, NZ, true>(s_p + (p / NY) * PLP + p % NY, NYP, s_tz);
    __syncthreads();
    for (int i = threadIdx.x; i < 6 * PL; i += NT) {
        const int c = i / PL, r = i - c * PL, z = r / NY, y = r - z * NY;
        buf[c * cs + (long)r * M + kx] = s_p[c * PLP + z * NYP + y];
    }
    if (want_inv) block_reduce_store<NT, INV_NPART>(acc, mem.partials + (long)kx * INV_NPART, s_red);
}

// The member's basic invariant record from its nparts partial records, by the first wave
// of a workgroup alone (no barrier, so any block size will do): per-lane compensated
// sums over records lane, lane + 64, ..., then a fixed butterfly across the lanes.  It
// writes the record finalize_member writes, its sums taken in another fixed order.
__device__ __forceinline__ void finalize_member_wave(const double* __restrict__ partials, int nparts,
                                                     double* __restrict__ out) {
    if (threadIdx.x >= 64) return;
    constexpr int Q = INV_NPART;
    double s[Q], c[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = c[q] = 0.0;
    for (int j = threadIdx.x; j < nparts; j += 64) {
        const double* rec = partials + (long)j * Q;
#pragma unroll
        for (int q = 0; q < Q; ++q) neumaier_add(s[q], c[q], rec[q]);
    }
#pragma unroll
    for (int q = 0; q < Q; ++q) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            const double os = __shfl_xor(s[q], off, 64), oc = __shfl_xor(c[q], off, 64);
            c[q] += oc;
            neumaier_add(s[q], c[q], os);
        }
    }
    if (threadIdx.x == 0) {
        out[0] = s[INV_E1] + c[INV_E1];
        out[1] = s[INV_H1] + c[INV_H1];
        out[2] = s[INV_M1X] + c[INV_M1X];
        out[3] = s[INV_M1Y] + c[INV_M1Y];
        out[4] = s[INV_M1Z] + c[INV_M1Z];
        out[5] = sqrt(s[INV_DIVH] + c[INV_DIVH]);
        out[6] = sqrt(s[INV_DIVE] + c[INV_DIVE]);
        out[7] = 0.0;
    }
}

// The x kernels of a plane step: the last workgroup (one past the row blocks) finalizes
// the member's nfin partial records, which the plane pass wrote; the others run the
// plain kernels' rows.
template <typename T, class P, int NP>
__global__ void __launch_bounds__(P::T * NP)
k_x_inv_fin(const MemberDesc<T>* __restrict__ md, long nrows, const cpx<T>* __restrict__ twx, int nfin) {
    if (blockIdx.x == gridDim.x - 1) {  // uniform per workgroup
        finalize_member_wave(md[blockIdx.y].partials, nfin, md[blockIdx.y].inv);
        return;
    }
    x_inv_body<T, P, NP>(md, nrows, twx);
}
template <typename T, class P, int NP>
__global__ void __launch_bounds__(P::T * NP)
k_x_invfwd_fin(const MemberDesc<T>* __restrict__ md, long nrows, const cpx<T>* __restrict__ twx, int nfin) {
    if (blockIdx.x == gridDim.x - 1) {
        finalize_member_wave(md[blockIdx.y].partials, nfin, md[blockIdx.y].inv);
        return;
    }
    x_invfwd_body<T, P, NP>(md, nrows, twx);
}

}  // namespace eifp
