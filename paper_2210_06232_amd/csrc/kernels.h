// kernels.h -- the five passes of one EI-FP time step and their helpers.
//
// State layout in HBM: six real components (Hx, Hy, Hz, Ex, Ey, Ez), each
// [Nz][Ny][Nx] with x fastest (the vector ordering of Sec. 2.2).  The transforms run
// in place on the same bytes viewed as [6][Nz][Ny][M] complex, M = Nx/2:
//
//   x pass   each row of Nx reals is a length-M complex FFT followed by the real-to-
//            complex split; the row then holds X[1..M-1] and, in slot 0, the packed pair
//            X[0] + i X[M].  The paper sets the Nyquist wavenumber to zero (Sec. 2.3),
//            so the kx = 0 and kx = Nx/2 planes see the same propagator; the packed
//            column is therefore propagated and transformed along y and z as one
//            complex column with no unpacking.
//   z pass   C2C along z, one component per workgroup, tiles of B adjacent x columns.
//   y pass   fused: C2C along y for all six components of a tile, the mode-wise
//            exponential propagator (Prop. 2.1/2.2, Alg. 2 step 4) with the 1/(Nx Ny Nz)
//            of the inverse transform folded in, the invariant partial sums, and the
//            inverse C2C along y.  Powers of two: one thread holds all six components
//            (k_fused; persistent workgroups in FP64, components transformed in pairs);
//            lengths with a factor 3: two thread groups hold H and E (k_fused_split).
//   z^-1, x^-1 as above in reverse (complex-to-real merge back).  Between two steps of
//            one call, x^-1 and the next x pass are one kernel (k_x_invfwd) that keeps
//            the physical row in registers: a call writes the state once, at its end.
//
// Every kernel works on a batch of solves of one shape ("members"): the member index
// comes from the grid and selects a descriptor (buffers and per-solve scalars) from a
// device array, so one launch advances every member of a batch.
#pragma once
#include "fft_core.h"

namespace eifp {

// Per-solve scalars of the fused pass (formed in FP64 on the host).
struct PropParams {
    double tau_s;          // tau / sqrt(mu eps)
    double tau_s_over_pi;  // tau / (pi sqrt(mu eps))
    double rh;             // sqrt(mu / eps): weight of i k x H^ in E^'
    double re;             // sqrt(eps / mu): weight of i k x E^ in H^'
    double inv_ns;         // 1 / (Nx Ny Nz)
    double nu[3];          // 2 pi / L_w
    double mu, eps;
    double inv_mu, inv_eps;
};

// One member of a batch.  state: the solve's six fields (x-forward source, x-inverse
// destination); work: the buffer the transforms run in (== state for a step, a scratch
// or anchor buffer for a forward-only transform); partials: ntiles records of
// INV_NPART doubles; inv: the finalized invariants (8 doubles); spec: the anchored
// spectrum a jump propagates from (unused otherwise).
template <typename T>
struct MemberDesc {
    cpx<T>* state;
    cpx<T>* work;
    double* partials;
    double* inv;
    const cpx<T>* spec;
    PropParams pp;
};

// invariant partial sums per workgroup (all in FP64); the extended record adds the
// energies of the derivatives and the second helicity (Thms 4.1 and 4.3)
enum { INV_E1 = 0, INV_H1, INV_M1X, INV_M1Y, INV_M1Z, INV_DIVH, INV_DIVE, INV_NPART = 8 };
enum { INV_E2 = 8, INV_E3X, INV_E3Y, INV_E3Z, INV_E4X, INV_E4Y, INV_E4Z, INV_H2 };
// and the sums behind the drift scales (Cauchy-Schwarz bounds of H1, M1, the divergence
// norms): sum |b| (|H|^2/(2 eps) + |E|^2/(2 mu)), sum |H|^2, sum b_k^2 |E|^2, sum |b|^2 |H|^2,
// sum |b|^2 |E|^2 (one slot unused)
enum { INV_SH1 = 16, INV_HH, INV_BEX, INV_BEY, INV_BEZ, INV_B2H, INV_B2E, INV_XPART = 24 };

// Omega_w[m] of Sec. 2.3: nu m for m < n/2, 0 at the Nyquist index, nu (m - n) above.
__device__ __forceinline__ double omega(int m, int n, double nu) {
    const int half = n >> 1;
    return m < half ? nu * (double)m : (m == half ? 0.0 : nu * (double)(m - n));
}

// ---------------------------------------------------------------------------------
// x pass: real <-> packed half spectrum along contiguous rows
// ---------------------------------------------------------------------------------
// Pass order through the state (EIFP_MALL_ORDER = 1): each pass starts with the data the
// pass before it wrote last, which is still in the 256 MB last-level cache.  x forward
// ascending rows -> z forward descending components -> fused y (reads every component
// of a tile) -> z inverse ascending components -> x inverse descending rows -> (next
// step) x forward ascending rows.
#ifndef EIFP_MALL_ORDER
#define EIFP_MALL_ORDER 1
#endif
// twx[k] = exp(-2 pi i k / Nx), k < Nx (the length-M FFT reads every second entry).
//
// Register index holding position block m (position t + T m) in first- or last-stage
// order: the inverses of m_first and m_last.
template <class P>
__host__ __device__ constexpr int reg_of(int m, bool last) {
    const int R = last ? P::R[P::S - 1] : P::R[0], W = P::E / R;
    return (m % W) * R + m / W;
}

// The value of lane l ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float swap_lane_pair(float x) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), 0xB1, 0xF, 0xF, false));
}

// Store a row held as v[i] at positions t + T m(i) (m = m_last if LAST, else m_first).
// With 8-byte elements and 8 threads per row a store instruction would cover half of
// each 128-byte line of the row, and the two halves would reach memory separately;
// instead lanes t and t ^ 1 trade one value so that each lane stores two adjacent
// elements (16 bytes) and one instruction covers blocks m and m + 1 (m even) of the row:
// whole lines.
template <typename T, class P, bool LAST>
__device__ __forceinline__ void store_row(cpx<T>* out, const cpx<T> (&v)[P::E], int t, bool active) {
    constexpr int E = P::E, TT = P::T;
    typedef T quad_t __attribute__((ext_vector_type(4)));
    if constexpr (sizeof(T) == 4 && TT == 8 && E % 2 == 0) {
        const bool odd = t & 1;
#pragma unroll
        for (int m = 0; m < E; m += 2) {
            const cpx<T> a = v[reg_of<P>(m, LAST)], b = v[reg_of<P>(m + 1, LAST)];
            const cpx<T> send = odd ? a : b;
            const cpx<T> recv = {swap_lane_pair(send.x), swap_lane_pair(send.y)};
            // even lane t: elements t, t + 1 of block m; odd lane t: elements t - 1, t of block m + 1
            const cpx<T> lo = odd ? recv : a, hi = odd ? b : recv;
            const int pos = odd ? TT * (m + 1) + t - 1 : TT * m + t;
            quad_t q;
            q.x = lo.x;
            q.y = lo.y;
            q.z = hi.x;
            q.w = hi.y;
            if (active) *reinterpret_cast<quad_t*>(out + pos) = q;
        }
    } else if (active) {
#pragma unroll
        for (int i = 0; i < E; ++i) out[t + TT * (LAST ? m_last<P>(i) : m_first<P>(i))] = v[i];
    }
}

// Row helpers.  x_forward_row: v holds the row's M complex values (pairs of reals) at
// positions t + T m_first(i); length-M FFT, then the split
//   X[k] = (Z[k] + conj Z[M-k])/2 - (i/2) W^k (Z[k] - conj Z[M-k]),  W = exp(-2 pi i/Nx),
// stored to out (X[0] + i X[M] in slot 0).  The row's LDS and the twiddle table are
// ordered by the caller (the table staged behind a block barrier).
template <typename T, class P, int LD>
__device__ __forceinline__ void x_forward_row(cpx<T> (&v)[P::E], int t, LdsRows<T, LD>& lds, const cpx<T>* s_tw,
                                              cpx<T>* out, bool active) {
    constexpr int M = P::N, E = P::E, TT = P::T;
    static_assert(64 % TT == 0, "a row within one wave");
    fft_pencil<P, false, 2>(v, t, lds, s_tw);
    lds.after_load();  // the row's last exchange read before it is written again
#pragma unroll
    for (int i = 0; i < E; ++i) lds.st(t + TT * m_last<P>(i), v[i]);
    lds.sync();
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int k = t + TT * m_last<P>(i);
        const cpx<T> z = v[i];
        if (k == 0) {
            v[i] = {z.x + z.y, z.x - z.y};  // X[0] + i X[M]
        } else {
            const cpx<T> zc = conj(lds.ld(M - k));
            const cpx<T> ev = scale(z + zc, (T)0.5);
            const cpx<T> od = scale(mulmi(z - zc), (T)0.5);  // (Z - conj Z')/(2i)
            v[i] = ev + twmul<false>(s_tw, k, 2 * M, od);
        }
    }
    store_row<T, P, true>(out, v, t, active);
}

// x_inverse_row: v holds the packed half spectrum of a row at positions t + T m_first(i);
// merge Z[k] = (X[k] + conj X[M-k]) + i W^-k (X[k] - conj X[M-k]) (Z[0] from X[0], X[M]),
// then the inverse length-M FFT: v ends at positions t + T m_last(i) (the row's reals in
// pairs, unscaled).
template <typename T, class P, int LD>
__device__ __forceinline__ void x_inverse_row(cpx<T> (&v)[P::E], int t, LdsRows<T, LD>& lds, const cpx<T>* s_tw) {
    constexpr int M = P::N, E = P::E, TT = P::T;
    static_assert(64 % TT == 0, "a row within one wave");
#pragma unroll
    for (int i = 0; i < E; ++i) lds.st(t + TT * m_first<P>(i), v[i]);
    lds.sync();
#pragma unroll
    for (int i = 0; i < E; ++i) {
        const int k = t + TT * m_first<P>(i);
        const cpx<T> x = v[i];
        if (k == 0) {
            v[i] = {x.x + x.y, x.x - x.y};
        } else {
            const cpx<T> xc = conj(lds.ld(M - k));
            v[i] = (x + xc) + muli(twmul<true>(s_tw, k, 2 * M, x - xc));
        }
    }
    lds.after_load();
    fft_pencil<P, true, 2>(v, t, lds, s_tw);
}

// Grid: (row blocks, members).  Forward reads state, writes work.
template <typename T, class P, int NP>
__global__ void __launch_bounds__(P::T * NP)
k_x_fwd(const MemberDesc<T>* __restrict__ md, long nrows, const cpx<T>* __restrict__ twx) {
    constexpr int M = P::N, E = P::E, TT = P::T, LD = rows_pitch<T>(M);
    __shared__ T s_re[NP * LD];
    __shared__ T s_im[NP * LD];
    __shared__ cpx<T> s_tw[2 * M * TwParts<T>::value];
    stage_table(s_tw, twx, 2 * M);
    __syncthreads();  // the table, before any wave's first use
    const cpx<T>* src = md[blockIdx.y].state;
    cpx<T>* dst = md[blockIdx.y].work;
    const int t = threadIdx.x % TT, p = threadIdx.x / TT;
    const long row = (long)blockIdx.x * NP + p;
    const bool active = row < nrows;
    // rows past the end read the last row (in bounds, never stored) instead of branching
    const cpx<T>* in = src + (active ? row : nrows - 1) * M;
    cpx<T> v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = in[t + TT * m_first<P>(i)];
    LdsRows<T, LD> lds{s_re, s_im, p};
    x_forward_row<T, P, LD>(v, t, lds, s_tw, dst + row * M, active);
}

// Rows in descending order (EIFP_MALL_ORDER): the z inverse pass wrote the last
// components last, and those are the ones still in the last-level cache.
__device__ __forceinline__ long x_inv_row(long nrows, int np, int p) {
    const long r = (long)blockIdx.x * np + p;
    return EIFP_MALL_ORDER ? nrows - 1 - r : r;
}

// Inverse reads work, writes state.  (The body is shared with k_x_inv_fin.)
template <typename T, class P, int NP>
__device__ __forceinline__ void x_inv_body(const MemberDesc<T>* __restrict__ md, long nrows,
                                           const cpx<T>* __restrict__ twx) {
    constexpr int M = P::N, E = P::E, TT = P::T, LD = rows_pitch<T>(M);
    __shared__ T s_re[NP * LD];
    __shared__ T s_im[NP * LD];
    __shared__ cpx<T> s_tw[2 * M * TwParts<T>::value];
    stage_table(s_tw, twx, 2 * M);
    __syncthreads();  // the table, before any wave's first use
    const cpx<T>* src = md[blockIdx.y].work;
    cpx<T>* dst = md[blockIdx.y].state;
    const int t = threadIdx.x % TT, p = threadIdx.x / TT;
    const long row = x_inv_row(nrows, NP, p);
    const bool active = row >= 0 && row < nrows;
    const cpx<T>* in = src + (active ? row : nrows - 1) * M;
    LdsRows<T, LD> lds{s_re, s_im, p};
    cpx<T> v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = in[t + TT * m_first<P>(i)];
    x_inverse_row<T, P, LD>(v, t, lds, s_tw);
    store_row<T, P, true>(dst + row * M, v, t, active);
}
template <typename T, class P, int NP>
__global__ void __launch_bounds__(P::T * NP)
k_x_inv(const MemberDesc<T>* __restrict__ md, long nrows, const cpx<T>* __restrict__ twx) {
    x_inv_body<T, P, NP>(md, nrows, twx);
}

// Between two steps (work != state): the x inverse of one step and the x forward of the
// next on the same row, in place on work (the spectrum after the z inverse).  The
// physical row, the state after this step, lives only in registers: within one call
// nothing reads an intermediate state (the invariants are summed in spectral space by
// the fused pass), and the call's last step ends with k_x_inv, which writes the state.
// The arithmetic is that of k_x_inv followed by k_x_fwd, with the physical row rounded
// to T as a store would round it, so a call of K steps gives the bits of K calls of one
// step, with one state read and one state write fewer per step.  Each row is read whole
// (before the first exchange barrier) by the threads that later write it.  Rows in the
// order of k_x_inv, so the z forward pass after it takes the components in ascending
// order.  (The body is shared with k_x_invfwd_fin.)
template <typename T, class P, int NP>
__device__ __forceinline__ void x_invfwd_body(const MemberDesc<T>* __restrict__ md, long nrows,
                                              const cpx<T>* __restrict__ twx) {
    constexpr int M = P::N, E = P::E, TT = P::T, LD = rows_pitch<T>(M);
    __shared__ T s_re[NP * LD];
    __shared__ T s_im[NP * LD];
    __shared__ cpx<T> s_tw[2 * M * TwParts<T>::value];
    stage_table(s_tw, twx, 2 * M);
    __syncthreads();  // the table, before any wave's first use
    cpx<T>* work = md[blockIdx.y].work;
    const int t = threadIdx.x % TT, p = threadIdx.x / TT;
    const long row = x_inv_row(nrows, NP, p);
    const bool active = row >= 0 && row < nrows;
    const cpx<T>* in = work + (active ? row : nrows - 1) * M;
    LdsRows<T, LD> lds{s_re, s_im, p};
    cpx<T> v[E];
#pragma unroll
    for (int i = 0; i < E; ++i) v[i] = in[t + TT * m_first<P>(i)];
    x_inverse_row<T, P, LD>(v, t, lds, s_tw);
    // the physical row as materialised values of T, as a store and a reload would give
    // them: the empty asm keeps the compiler from merging the inverse's last operations
    // with the forward's first ones (without it, FP64 rows differ in the last bit from
    // those of k_x_inv followed by k_x_fwd)
#pragma unroll
    for (int i = 0; i < E; ++i) asm volatile("" : "+v"(v[i].x), "+v"(v[i].y));
    last_to_first<P>(v);
    x_forward_row<T, P, LD>(v, t, lds, s_tw, work + row * M, active);
}
template <typename T, class P, int NP>
__global__ void __launch_bounds__(P::T * NP)
k_x_invfwd(const MemberDesc<T>* __restrict__ md, long nrows, const cpx<T>* __restrict__ twx) {
    x_invfwd_body<T, P, NP>(md, nrows, twx);
}

// ---------------------------------------------------------------------------------
// column access: tiles of B adjacent x columns, a pencil per column
// ---------------------------------------------------------------------------------
// Lane (c, t) of a tile owns column x0 + c and pencil positions t + T m.  Byte offsets
// are 32-bit: the lane part goes in a VGPR, the position part m T stride (wave-uniform)
// in the scalar offset of a raw buffer access.  Lanes past the last column load the
// last column (in bounds, never stored) so that loads need no branch.
template <typename T, class P>
__device__ __forceinline__ void load_col(cpx<T> (&v)[P::E], __amdgpu_buffer_rsrc_t r, unsigned voff, unsigned sstep) {
#pragma unroll
    for (int i = 0; i < P::E; ++i) v[i] = BufIO<T>::ld(r, voff, (unsigned)m_first<P>(i) * sstep);
}

// Cache policy of the column stores (the buffer store's cache-policy operand; 2 = the
// non-temporal hint).  The z passes store non-temporally when the state is larger than
// the last-level cache can usefully hold (the launcher's choice, the same bound as the
// x kernel's streaming stores): their output then streams past the caches, which takes
// ~6% off the z inverse at 256^3 (FP64) for ~2% on the x kernel that reads it next, ~1%
// per step in both forms.  The fused pass keeps the default (non-temporal stores cost
// it 6%).
#ifndef EIFP_FUSED_ST_AUX
#define EIFP_FUSED_ST_AUX 0
#endif
constexpr int kStoreNT = 2;
template <typename T, class P, int AUX = 0>
__device__ __forceinline__ void store_col(const cpx<T> (&v)[P::E], __amdgpu_buffer_rsrc_t r, unsigned voff,
                                          unsigned sstep, bool active) {
    if (active) {
#pragma unroll
        for (int i = 0; i < P::E; ++i) BufIO<T>::template st<AUX>(v[i], r, voff, (unsigned)m_last<P>(i) * sstep);
    }
}

// ---------------------------------------------------------------------------------
// deterministic compensated finalize of the invariant partials
// ---------------------------------------------------------------------------------
// Grid: one block per member.  out (member's inv): [0] E1 [1] H1 [2..4] M1
// [5] ||div~(mu H)||_N [6] ||div~(eps E)||_N; extended record: [8] E2 [9..11] E3
// [12..14] E4 [15] H2
__device__ __forceinline__ void neumaier_add(double& s, double& c, double x) {
    const double t = s + x;
    c += fabs(s) >= fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
}

// Thread j sums records j, j + 1024, ... (each record: Q contiguous doubles) with
// Neumaier compensation, then the 1024 (sum, compensation) pairs are combined by a
// fixed xor-butterfly inside each wave and a fixed loop over the 16 waves: the same
// partials always give the same bits.
// One member: thread j of the NT-thread workgroup sums records j, j + NT, ... (each
// record: Q contiguous doubles) with Neumaier compensation, then the (sum,
// compensation) pairs are combined by a fixed xor-butterfly inside each wave and a
// fixed loop over the waves: the same partials always give the same bits.  s_w holds
// 2 Q doubles per wave.
template <int Q, int NT>
__device__ __forceinline__ void finalize_member(const double* __restrict__ partials, int nparts, double* __restrict__ out,
                                                double* s_w) {
    static_assert(NT % 64 == 0, "whole waves");
    constexpr int NW = NT / 64;
    double s[Q], c[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) s[q] = c[q] = 0.0;
#pragma unroll 2
    for (int j = threadIdx.x; j < nparts; j += NT) {
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
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            s_w[wid * 2 * Q + q] = s[q];
            s_w[wid * 2 * Q + Q + q] = c[q];
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double res[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            double a = 0.0, ca = 0.0;
            for (int w = 0; w < NW; ++w) {
                ca += s_w[w * 2 * Q + Q + q];
                neumaier_add(a, ca, s_w[w * 2 * Q + q]);
            }
            res[q] = a + ca;
        }
        out[0] = res[INV_E1];
        out[1] = res[INV_H1];
        out[2] = res[INV_M1X];
        out[3] = res[INV_M1Y];
        out[4] = res[INV_M1Z];
        out[5] = sqrt(res[INV_DIVH]);
        out[6] = sqrt(res[INV_DIVE]);
        out[7] = 0.0;
#pragma unroll
        for (int q = INV_NPART; q < Q; ++q) out[q] = res[q];
    }
}

// Grid: one 1024-thread workgroup per member.
template <typename T, int Q>
__global__ void __launch_bounds__(1024) k_finalize(const MemberDesc<T>* __restrict__ md, int nparts) {
    __shared__ double s_w[16 * 2 * Q];
    finalize_member<Q, 1024>(md[blockIdx.x].partials, nparts, md[blockIdx.x].inv, s_w);
}

// ---------------------------------------------------------------------------------
// tile numbering
// ---------------------------------------------------------------------------------
// The dispatcher deals workgroups to the 8 XCDs round robin by linear id, and each XCD
// has its own L2.  With `on`, (blockIdx.x, blockIdx.y) are renumbered so that the
// workgroups one XCD receives (linear ids congruent mod 8) cover a contiguous range of
// tiles: neighbouring tiles, which share cache lines and DRAM pages, then run on the
// same XCD at about the same time.  nxt: tile columns (blockIdx.x < nxt).  A bijection
// whenever nxt * gridDim.y is a multiple of 8 (otherwise the ids are left as they are).
#ifndef EIFP_FUSED_XCD
#define EIFP_FUSED_XCD 1
#endif
#ifndef EIFP_C2C_XCD
#define EIFP_C2C_XCD 0
#endif
__device__ __forceinline__ void xcd_tiles(bool on, unsigned nxt, int& tx, int& ty) {
    tx = (int)blockIdx.x;
    ty = (int)blockIdx.y;
    const unsigned n = nxt * gridDim.y;
    if (!on || (n & 7u) != 0) return;
    const unsigned L = blockIdx.x + nxt * blockIdx.y;
    const unsigned Lp = (L & 7u) * (n >> 3) + (L >> 3);
    tx = (int)(Lp % nxt);
    ty = (int)(Lp / nxt);
}

// ---------------------------------------------------------------------------------
// single-component C2C pass along a strided axis (y or z), one component per workgroup
// ---------------------------------------------------------------------------------
// Pencil positions are pstride apart; the third (outer) axis index blockIdx.y is ostride
// apart; cs is the component stride; all in complex elements.  Grid: (x tiles, outer,
// 6 x members); runs in place on work.  With fin_nparts > 0 the grid has one more tile
// column, whose workgroup at outer index 0 and component 0 finalizes its member's
// invariant partials (fin_nparts records) while the other workgroups transform: the
// partials were written by the preceding fused pass, and the next one runs after this.
// The strided pass's exchange: unpadded rows skewed every 2^EIFP_CSKEW positions
// (EIFP_CSKEW = 1: log2 of the plan's first radix; 0: rows padded by EIFP_LDS_PAD), and
// stage twiddles in the plan's stage order (EIFP_C2C_STW).
#ifndef EIFP_CSKEW
#define EIFP_CSKEW 0
#endif
#ifndef EIFP_C2C_STW
#define EIFP_C2C_STW 1
#endif
template <class P>
__host__ __device__ constexpr int c2c_skew() {
    if (EIFP_CSKEW != 1) return EIFP_CSKEW;
    int k = 0;
    while ((1 << k) < P::R[0]) ++k;
    return k;
}
template <typename T, class P, int B, bool INV, int ST_AUX = 0>
__global__ void __launch_bounds__(P::T * B)
k_c2c(const MemberDesc<T>* __restrict__ md, int M, long pstride, long ostride, long cs,
      const cpx<T>* __restrict__ tw, int fin_nparts, int comp_desc) {
    constexpr int NP = P::N, E = P::E, TT = P::T;
    __shared__ double s_w[((TT * B + 63) / 64) * 2 * INV_NPART];
    const unsigned nxt = gridDim.x - (fin_nparts > 0 ? 1u : 0u);
    if (blockIdx.x >= nxt) {  // the finalize column (uniform per workgroup)
        if (blockIdx.y == 0 && blockIdx.z % 6 == 0) {
            const MemberDesc<T>& m = md[blockIdx.z / 6];
            finalize_member<INV_NPART, TT * B>(m.partials, fin_nparts, m.inv, s_w);
        }
        return;
    }
    constexpr int SK = c2c_skew<P>(), PITCH = SK > 0 ? B : col_pitch(B), ROWS = skew_rows<NP, SK>();
    __shared__ T s_re[ROWS * PITCH];
    __shared__ T s_im[ROWS * PITCH];
    __shared__ cpx<T> s_tw[NP * TwParts<T>::value];
    if (EIFP_C2C_STW) stage_table_plan<P>(s_tw, tw);
    else stage_table(s_tw, tw, NP);
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    int tx, ty;
    xcd_tiles(EIFP_C2C_XCD, nxt, tx, ty);
    const int col = tx * B + c;
    const int o = ty;
    // comp_desc: the components in descending order (EIFP_MALL_ORDER), for a forward
    // pass after k_x_fwd, which wrote the last components last (they are still in the
    // last-level cache); ascending after k_x_invfwd and for the inverse (so the x
    // inverse after it starts from the last component)
    const int member = blockIdx.z / 6;
    const int comp = (EIFP_MALL_ORDER && comp_desc) ? 5 - (int)(blockIdx.z % 6) : (int)(blockIdx.z % 6);
    const bool active = col < M;
    const __amdgpu_buffer_rsrc_t r = make_rsrc(md[member].work + comp * cs, (unsigned)(cs * sizeof(cpx<T>)));
    const unsigned voff = (unsigned)(t * pstride + o * ostride + (active ? col : M - 1)) * sizeof(cpx<T>);
    const unsigned sstep = (unsigned)(TT * pstride) * sizeof(cpx<T>);
    cpx<T> v[E];
    load_col<T, P>(v, r, voff, sstep);
    LdsCols<T, B, PITCH, SK> lds{s_re, s_im, c};
    fft_pencil<P, INV, EIFP_C2C_STW ? kStagedTw : 1>(v, t, lds, s_tw);
    store_col<T, P, ST_AUX>(v, r, voff, sstep, active);
}

// ---------------------------------------------------------------------------------
// fused pass: forward, propagate, invariant partials, inverse (all six components)
// ---------------------------------------------------------------------------------
// Z_STEP: forward, propagate by the member's tau, partials, inverse (one time step).
// Z_FORWARD: forward, partials only (invariants of the state; memory untouched).
// Z_JUMP: read the anchored spectrum (all three forward transforms already done),
// propagate by the member's tau, partials, inverse along the fused axis into work.
// Z_FORWARD_EXT: as Z_FORWARD with the extended invariant record.
enum ZMode { Z_STEP = 0, Z_FORWARD = 1, Z_JUMP = 2, Z_FORWARD_EXT = 3 };
template <int MODE> struct NQ { static constexpr int value = MODE == Z_FORWARD_EXT ? INV_XPART : INV_NPART; };

template <typename T>
__device__ __forceinline__ double dreal(T a) { return (double)a; }

// Accumulate the weighted spectral sums of one mode.  h, e are the six propagated
// coefficients already multiplied by 1/N_S, so sums of their products are the
// discrete inner products of Sec. 4 (Parseval) with no further scaling.
template <int Q, typename T>
__device__ __forceinline__ void accumulate_invariants(double (&acc)[Q], double w, double bx, double by, double bz,
                                                      const cpx<T>* h, const cpx<T>* e, const PropParams& pp) {
    const double mu = pp.mu, eps = pp.eps;
    const double hr[3] = {dreal(h[0].x), dreal(h[1].x), dreal(h[2].x)};
    const double hi[3] = {dreal(h[0].y), dreal(h[1].y), dreal(h[2].y)};
    const double er[3] = {dreal(e[0].x), dreal(e[1].x), dreal(e[2].x)};
    const double ei[3] = {dreal(e[0].y), dreal(e[1].y), dreal(e[2].y)};
    double h2 = 0, e2 = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        h2 += hr[c] * hr[c] + hi[c] * hi[c];
        e2 += er[c] * er[c] + ei[c] * ei[c];
    }
    acc[INV_E1] += w * 0.5 * (mu * h2 + eps * e2);
    // b . (Re U x Im U)
    const double hc = bx * (hr[1] * hi[2] - hr[2] * hi[1]) + by * (hr[2] * hi[0] - hr[0] * hi[2]) +
                      bz * (hr[0] * hi[1] - hr[1] * hi[0]);
    const double ec = bx * (er[1] * ei[2] - er[2] * ei[1]) + by * (er[2] * ei[0] - er[0] * ei[2]) +
                      bz * (er[0] * ei[1] - er[1] * ei[0]);
    acc[INV_H1] += w * (hc * pp.inv_eps + ec * pp.inv_mu);
    // Im H . Re E - Re H . Im E
    double q = 0;
#pragma unroll
    for (int c = 0; c < 3; ++c) q += hi[c] * er[c] - hr[c] * ei[c];
    acc[INV_M1X] += w * bx * q;
    acc[INV_M1Y] += w * by * q;
    acc[INV_M1Z] += w * bz * q;
    const double dhr = bx * hr[0] + by * hr[1] + bz * hr[2], dhi = bx * hi[0] + by * hi[1] + bz * hi[2];
    const double der = bx * er[0] + by * er[1] + bz * er[2], dei = bx * ei[0] + by * ei[1] + bz * ei[2];
    acc[INV_DIVH] += w * mu * mu * (dhr * dhr + dhi * dhi);
    acc[INV_DIVE] += w * eps * eps * (der * der + dei * dei);
    if constexpr (Q > INV_NPART) {
        // time derivatives from the semi-discrete system: d/dt H^ = -(i/mu) b x E^,
        // d/dt E^ = (i/eps) b x H^, with |b x U|^2 = |b|^2 |U|^2 - |b . U|^2 and
        // b . (Re(b x A) x Re(b x B))-type helicity terms equal to |b|^2 times the
        // undifferentiated ones
        const double b2 = bx * bx + by * by + bz * bz;
        const double en1 = 0.5 * (mu * h2 + eps * e2);
        const double en2 = 0.5 * pp.inv_mu * (b2 * e2 - (der * der + dei * dei)) +
                           0.5 * pp.inv_eps * (b2 * h2 - (dhr * dhr + dhi * dhi));
        acc[INV_E2] += w * en2;
        const double bk2[3] = {bx * bx, by * by, bz * bz};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            acc[INV_E3X + k] += w * bk2[k] * en1;
            acc[INV_E4X + k] += w * bk2[k] * en2;
        }
        acc[INV_H2] += w * b2 * pp.inv_mu * pp.inv_eps * (hc * pp.inv_eps + ec * pp.inv_mu);
        acc[INV_SH1] += w * sqrt(b2) * 0.5 * (h2 * pp.inv_eps + e2 * pp.inv_mu);
        acc[INV_HH] += w * h2;
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[INV_BEX + k] += w * bk2[k] * e2;
        acc[INV_B2H] += w * b2 * h2;
        acc[INV_B2E] += w * b2 * e2;
    }
}

// Block-wide sum of Q doubles in a fixed order; thread 0 writes the partials.
template <int NT, int Q>
__device__ __forceinline__ void block_reduce_store(double (&acc)[Q], double* __restrict__ out, double* s_red) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        double a = acc[q];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off, 64);
        acc[q] = a;
    }
    constexpr int NW = (NT + 63) / 64;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) s_red[wid * Q + q] = acc[q];
    }
    __syncthreads();
    if (threadIdx.x < Q) {
        double a = 0;
        for (int w = 0; w < NW; ++w) a += s_red[w * Q + threadIdx.x];
        out[threadIdx.x] = a;
    }
}

// sin(pi x) and cos(pi x) in FP64, from the Taylor series of sin and cos: x = n/2 + r with
// n = rint(2x) and |r| <= 1/4 (n/2 and r are exact in FP64), sin(pi r) and cos(pi r) by
// Horner in r^2 through the terms of degree 17 and 16 (the first terms left out are below
// 1e-19 and 3e-18 at |r| = 1/4), then the n mod 4 quarter turns.  About half the
// instructions of the library's sincospi, within a couple of units in the last place.
#ifndef EIFP_SERIES_SINCOS
#define EIFP_SERIES_SINCOS 1
#endif
__host__ __device__ inline void sincospi_series(double x, double* sn, double* cs) {
    const double n = rint(2.0 * x);
    const double r = fma(-0.5, n, x);
    const double z = r * r;
    // (-1)^k pi^(2k+1) / (2k+1)!, k = 8 .. 0
    double ps = 7.952054001475513e-07;
    ps = fma(ps, z, -2.1915353447830217e-05);
    ps = fma(ps, z, 0.00046630280576761255);
    ps = fma(ps, z, -0.0073704309457143504);
    ps = fma(ps, z, 0.08214588661112823);
    ps = fma(ps, z, -0.5992645293207921);
    ps = fma(ps, z, 2.5501640398773455);
    ps = fma(ps, z, -5.16771278004997);
    ps = fma(ps, z, 3.141592653589793);
    // (-1)^k pi^(2k) / (2k)!, k = 8 .. 0
    double pc = 4.303069587032947e-06;
    pc = fma(pc, z, -0.0001046381049248457);
    pc = fma(pc, z, 0.0019295743094039231);
    pc = fma(pc, z, -0.02580689139001406);
    pc = fma(pc, z, 0.2353306303588932);
    pc = fma(pc, z, -1.3352627688545895);
    pc = fma(pc, z, 4.0587121264167685);
    pc = fma(pc, z, -4.934802200544679);
    pc = fma(pc, z, 1.0);
    const double s = r * ps, c = pc;
    const int q = (int)(n - 4.0 * floor(0.25 * n));  // n mod 4, exact
    const double so = (q & 1) ? c : s, co = (q & 1) ? s : c;
    *sn = q >= 2 ? -so : so;
    *cs = (q == 1 || q == 2) ? -co : co;
}

// Propagate one mode in place.  b = (Omega_x, Omega_y, Omega_z).  With k = b/|b|,
// theta = tau |b| / sqrt(mu eps), L(U) = k (k.U), X(U) = i k x U:
//   H' = L(H) + cos(theta) (H - L(H)) - sin(theta) sqrt(eps/mu) X(E)
//   E' = L(E) + cos(theta) (E - L(E)) + sin(theta) sqrt(mu/eps) X(H)
// which is the c/s matrix of Prop. 2.2 applied as in Alg. 2 step 4 (c = k k^T +
// cos(theta) (I - k k^T), s_12 = i sin(theta) k_z, ...).  |b| = 0 keeps the mode.
// All coefficients are formed in FP64 and rounded to T; everything is scaled by 1/N_S.
#ifndef EIFP_PROP_COMP
#define EIFP_PROP_COMP 1
#endif
template <typename T>
__device__ __forceinline__ void propagate_mode(cpx<T>* h, cpx<T>* e, double bx, double by, double bz, const PropParams& pp) {
    // |b| = 0 needs no branch: theta = 0 gives cos = 1, sin = 0 and the k terms drop out
    const double b2 = bx * bx + by * by + bz * bz;
    const double ib = b2 > 0.0 ? rsqrt(b2) : 0.0;  // 1/|b| (0 for the zero mode)
    const double bn = b2 * ib;                      // |b|
    // the phase in half-turns, theta / pi, so that the reduction is exact for any tau
    double sn, cs;
    if (EIFP_SERIES_SINCOS) sincospi_series(pp.tau_s_over_pi * bn, &sn, &cs);
    else sincospi(pp.tau_s_over_pi * bn, &sn, &cs);
    if constexpr (sizeof(T) == 4 && EIFP_PROP_COMP) {
        // FP32: every coefficient of the transverse rotation (cos, sin, the unit wave
        // vector in the cross products) enters as a rounded part plus its remainder,
        // folded into the FMA chain before the final rounding, so the per-mode rotation
        // is not biased in modulus from step to step
        const double kd[3] = {bx * ib, by * ib, bz * ib};
        float kh_[3], kl_[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            kh_[c] = (float)kd[c];
            kl_[c] = (float)(kd[c] - (double)kh_[c]);
        }
        const double cTd = cs * pp.inv_ns, sEd = sn * pp.re * pp.inv_ns, sHd = sn * pp.rh * pp.inv_ns;
        const float cTh = (float)cTd, cTl = (float)(cTd - (double)cTh);
        const float sEh = (float)sEd, sEl = (float)(sEd - (double)sEh);
        const float sHh = (float)sHd, sHl = (float)(sHd - (double)sHh);
        const float dL = (float)((1.0 - cs) * pp.inv_ns);
        const cpx<float> kh = {kh_[0] * (float)h[0].x + kh_[1] * (float)h[1].x + kh_[2] * (float)h[2].x,
                               kh_[0] * (float)h[0].y + kh_[1] * (float)h[1].y + kh_[2] * (float)h[2].y};
        const cpx<float> ke = {kh_[0] * (float)e[0].x + kh_[1] * (float)e[1].x + kh_[2] * (float)e[2].x,
                               kh_[0] * (float)e[0].y + kh_[1] * (float)e[1].y + kh_[2] * (float)e[2].y};
        // (k x U)_c = k_a U_b - k_b U_a with (a, b) = (y, z), (z, x), (x, y)
        auto cross = [&](const float* ur, int c) {
            const int a = (c + 1) % 3, b = (c + 2) % 3;
            return __builtin_fmaf(kh_[a], ur[b],
                                  __builtin_fmaf(-kh_[b], ur[a], __builtin_fmaf(kl_[a], ur[b], -(kl_[b] * ur[a]))));
        };
        const float her[3] = {(float)h[0].x, (float)h[1].x, (float)h[2].x}, hei[3] = {(float)h[0].y, (float)h[1].y, (float)h[2].y};
        const float eer[3] = {(float)e[0].x, (float)e[1].x, (float)e[2].x}, eei[3] = {(float)e[0].y, (float)e[1].y, (float)e[2].y};
        float xer[3], xei[3], xhr[3], xhi[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xer[c] = cross(eer, c);
            xei[c] = cross(eei, c);
            xhr[c] = cross(her, c);
            xhi[c] = cross(hei, c);
        }
        // H' = cT H + dL k (k.H) - sE i (k x E);  E' = cT E + dL k (k.E) + sH i (k x H);  i (a + ib) = -b + ia
        auto comb = [&](float u, float x, float lon, float sh, float sl) {
            return __builtin_fmaf(cTh, u, __builtin_fmaf(sh, x, __builtin_fmaf(cTl, u, __builtin_fmaf(sl, x, lon))));
        };
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float dk = dL * kh_[c];
            const cpx<float> hn = {comb(her[c], xei[c], dk * kh.x, sEh, sEl), comb(hei[c], -xer[c], dk * kh.y, sEh, sEl)};
            const cpx<float> en = {comb(eer[c], -xhi[c], dk * ke.x, sHh, sHl), comb(eei[c], xhr[c], dk * ke.y, sHh, sHl)};
            h[c] = {(T)hn.x, (T)hn.y};
            e[c] = {(T)en.x, (T)en.y};
        }
        return;
    }
    const T kx = (T)(bx * ib), ky = (T)(by * ib), kz = (T)(bz * ib);
    const T cT = (T)(cs * pp.inv_ns);                 // transverse part
    const T dL = (T)((1.0 - cs) * pp.inv_ns);         // longitudinal minus transverse
    const T sE = (T)(sn * pp.re * pp.inv_ns);
    const T sH = (T)(sn * pp.rh * pp.inv_ns);
    const cpx<T> kh = {kx * h[0].x + ky * h[1].x + kz * h[2].x, kx * h[0].y + ky * h[1].y + kz * h[2].y};
    const cpx<T> ke = {kx * e[0].x + ky * e[1].x + kz * e[2].x, kx * e[0].y + ky * e[1].y + kz * e[2].y};
    // k x U
    const cpx<T> xe[3] = {{ky * e[2].x - kz * e[1].x, ky * e[2].y - kz * e[1].y},
                          {kz * e[0].x - kx * e[2].x, kz * e[0].y - kx * e[2].y},
                          {kx * e[1].x - ky * e[0].x, kx * e[1].y - ky * e[0].y}};
    const cpx<T> xh[3] = {{ky * h[2].x - kz * h[1].x, ky * h[2].y - kz * h[1].y},
                          {kz * h[0].x - kx * h[2].x, kz * h[0].y - kx * h[2].y},
                          {kx * h[1].x - ky * h[0].x, kx * h[1].y - ky * h[0].y}};
    const T kk[3] = {kx, ky, kz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // i (k x E) = (-Im, Re)
        const cpx<T> hn = {cT * h[c].x + dL * kk[c] * kh.x + sE * xe[c].y, cT * h[c].y + dL * kk[c] * kh.y - sE * xe[c].x};
        const cpx<T> en = {cT * e[c].x + dL * kk[c] * ke.x - sH * xh[c].y, cT * e[c].y + dL * kk[c] * ke.y + sH * xh[c].x};
        h[c] = hn;
        e[c] = en;
    }
}

// Per-thread sums of the basic invariants along one y pencil.  The thread's column (so
// b_x and the packed-column weight) and its z index (b_z) are fixed, so only the terms
// that vary along the pencil are summed per mode; b_x, b_z, the weight and the
// material factors are applied once, in finish().
struct PencilSums {
    double h2 = 0, e2 = 0;               // |H|^2, |E|^2
    double chx = 0, chy = 0, chz = 0;    // (Re H x Im H)_x, b_y (..)_y, (..)_z
    double cex = 0, cey = 0, cez = 0;    // the same for E
    double q = 0, qy = 0;                // Im H . Re E - Re H . Im E, and b_y times it
    double dh = 0, de = 0;               // |b . H|^2, |b . E|^2
    template <typename T>
    __device__ __forceinline__ void add(double bx, double by, double bz, const cpx<T>* h, const cpx<T>* e) {
        const double hr[3] = {dreal(h[0].x), dreal(h[1].x), dreal(h[2].x)};
        const double hi[3] = {dreal(h[0].y), dreal(h[1].y), dreal(h[2].y)};
        const double er[3] = {dreal(e[0].x), dreal(e[1].x), dreal(e[2].x)};
        const double ei[3] = {dreal(e[0].y), dreal(e[1].y), dreal(e[2].y)};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            h2 += hr[c] * hr[c] + hi[c] * hi[c];
            e2 += er[c] * er[c] + ei[c] * ei[c];
        }
        chx += hr[1] * hi[2] - hr[2] * hi[1];
        chy += by * (hr[2] * hi[0] - hr[0] * hi[2]);
        chz += hr[0] * hi[1] - hr[1] * hi[0];
        cex += er[1] * ei[2] - er[2] * ei[1];
        cey += by * (er[2] * ei[0] - er[0] * ei[2]);
        cez += er[0] * ei[1] - er[1] * ei[0];
        double qq = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) qq += hi[c] * er[c] - hr[c] * ei[c];
        q += qq;
        qy += by * qq;
        const double dhr = bx * hr[0] + by * hr[1] + bz * hr[2], dhi = bx * hi[0] + by * hi[1] + bz * hi[2];
        const double der = bx * er[0] + by * er[1] + bz * er[2], dei = bx * ei[0] + by * ei[1] + bz * ei[2];
        dh += dhr * dhr + dhi * dhi;
        de += der * der + dei * dei;
    }
    __device__ __forceinline__ void finish(double (&acc)[INV_NPART], double w, double bx, double bz,
                                           const PropParams& pp) const {
        acc[INV_E1] = w * 0.5 * (pp.mu * h2 + pp.eps * e2);
        acc[INV_H1] = w * ((bx * chx + chy + bz * chz) * pp.inv_eps + (bx * cex + cey + bz * cez) * pp.inv_mu);
        acc[INV_M1X] = w * bx * q;
        acc[INV_M1Y] = w * qy;
        acc[INV_M1Z] = w * bz * q;
        acc[INV_DIVH] = w * pp.mu * pp.mu * dh;
        acc[INV_DIVE] = w * pp.eps * pp.eps * de;
        acc[INV_DIVE + 1] = 0.0;
    }
};

// Minimum waves per SIMD requested for the fused kernel (caps its register budget).
#ifndef EIFP_ZWAVES64
#define EIFP_ZWAVES64 1
#endif
#ifndef EIFP_ZWAVES32
#define EIFP_ZWAVES32 2
#endif
template <typename T, int N> struct ZWaves {
    // lengths with a factor 3 (6 values per thread in FP64, 12 in FP32): one wave
    static constexpr int value = (N % 3 == 0) ? 1 : (sizeof(T) == 8 ? EIFP_ZWAVES64 : EIFP_ZWAVES32);
};

// Which FFT stages of the fused pass use the FP32 tables' compensation terms (bit s =
// stage s; -1 = all).  Uncompensated, the first twiddled stage alone (the 64th or 48th
// roots of unity, whose FP32 roundings are biased low in modulus) costs about a third
// of a unit roundoff of energy per transform, so an FP32 run's energy drifts linearly
// and its error grows linearly; compensated, the error grows like the square root of
// the step count.  All stages cost ~6% on the FP32 fused pass, without spills.
#ifndef EIFP_FUSED_CT
#define EIFP_FUSED_CT -1
#endif

// scheduling fences of the fused pass: bit 0 between components' transforms, bit 1
// between modes of the propagator
#ifndef EIFP_FUSED_SB
#define EIFP_FUSED_SB 3
#endif

// The fused pass transforms, propagates and transforms back along one strided axis.
// AXIS = 1: pencils along y (stride M), one tile row per z index; AXIS = 2: pencils along
// z (stride Ny M), one tile row per y index.  Strides in complex elements; cs is the
// component stride.  The ntx x n_outer tiles of a member are shared by gridDim.x
// workgroups (grid: (G, 1, members)), each taking tiles in turn (persist_tile); the
// loads of a workgroup's next tile are issued component by component as the inverse
// transforms of the current tile store theirs, into the registers just freed, so they
// overlap the rest of the tile's work.  Each workgroup writes one partial record, at
// index blockIdx.x of its member's partials, summed over its tiles in a fixed order.
//
// Tile of work item k of workgroup g: the dispatcher deals workgroups to the 8 XCDs
// round robin, so with G a multiple of 8 the workgroups of one XCD take a contiguous
// block of G/8 tiles at every k (neighbouring tiles share cache lines).
__device__ __forceinline__ int persist_tile(int k, int G) {
    const int g = (int)blockIdx.x;
    if ((G & 7) != 0 || !EIFP_FUSED_XCD) return k * G + g;
    return k * G + (g & 7) * (G >> 3) + (g >> 3);
}

// Persistent workgroups (with the prefetch of the next tile) in FP64; in FP32 the loop's
// extra live registers spill at two waves per SIMD, so each workgroup takes one tile.
#ifndef EIFP_ZPERSIST64
#define EIFP_ZPERSIST64 1
#endif
#ifndef EIFP_ZPERSIST32
#define EIFP_ZPERSIST32 0
#endif
// Components transformed in lockstep by the fused pass (1, 2, 3 or 6): they share each
// exchange's barrier; their double-buffered exchange takes 4 NC N' B sizeof(T) bytes.
#ifndef EIFP_ZLOCK64
#define EIFP_ZLOCK64 2
#endif
#ifndef EIFP_ZLOCK32
#define EIFP_ZLOCK32 2
#endif
template <typename T, int N> struct ZLockstep {
    // (one at a time for lengths with a factor 3, and above 256, where the LDS of two
    // workgroups per CU would not hold them)
    static constexpr int value = (N % 3 == 0 || N > 256) ? 1 : (sizeof(T) == 8 ? EIFP_ZLOCK64 : EIFP_ZLOCK32);
};
// Persistent fused pass: drain the vector memory counter between the last component
// group's stores and its next-tile loads (256^3 FP64: fused pass 0.426-0.429 -> 0.419-0.420
// ms; a drain after every group, or stores before loads in every group without it, are
// slower; the split pass at 192^3 is unchanged by it and has none)
#ifndef EIFP_FUSED_DRAIN
#define EIFP_FUSED_DRAIN 1
#endif
template <typename T> struct ZPersist {
    static constexpr bool value = sizeof(T) == 8 ? EIFP_ZPERSIST64 != 0 : EIFP_ZPERSIST32 != 0;
};

template <typename T, class P, int B, int MODE, int AXIS>
__global__ void __launch_bounds__(P::T * B, (ZWaves<T, P::N>::value))
k_fused(const MemberDesc<T>* __restrict__ md, int M, int n_outer, int ntx, long pstride, long ostride, long cs,
        const cpx<T>* __restrict__ tw, int want_inv) {
    constexpr bool PERSIST = ZPersist<T>::value;
    constexpr int NZ = P::N, E = P::E, TT = P::T, NT = P::T * B;
    constexpr int PLANE = zplane<P, B>();
    constexpr int NC = ZLockstep<T, P::N>::value;  // components transformed together
    static_assert(6 % NC == 0, "components in equal groups");
    __shared__ T s_x[2 * 2 * NC * PLANE];
    __shared__ cpx<T> s_tw[NZ * TwParts<T>::value];
    constexpr int Q = NQ<MODE>::value;
    __shared__ double s_red[((NT + 63) / 64) * Q];
    stage_table_plan<P>(s_tw, tw);  // ordered by stage (conflict-free reads)
    const MemberDesc<T>& mem = md[blockIdx.z];
    const PropParams pp = mem.pp;
    cpx<T>* buf = mem.work;
    const cpx<T>* src = MODE == Z_JUMP ? mem.spec : buf;
    const int c = threadIdx.x % B, t = threadIdx.x / B;
    const int G = (int)gridDim.x, ntiles = ntx * n_outer;
    const unsigned cbytes = (unsigned)cs * sizeof(cpx<T>);
    const unsigned sstep = (unsigned)(TT * pstride) * sizeof(cpx<T>);
    LdsColsN<T, B, PLANE, zcol_pitch(B), zskew<P>(), NC> lds{s_x, c, 0};
    // per-tile geometry: the column, the outer index, and this lane's base offset
    struct Tile {
        int col, o;
        bool active;
        unsigned voff;
    };
    auto tile = [&](int w) {
        Tile a;
        a.col = (w % ntx) * B + c;
        a.o = w / ntx;
        a.active = a.col < M;
        a.voff = (unsigned)(t * pstride + a.o * ostride + (a.active ? a.col : M - 1)) * sizeof(cpx<T>);
        return a;
    };

    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    int k = 0;
    int wk = persist_tile(0, G);
    Tile cur = tile(wk < ntiles ? wk : 0);
    cpx<T> v[6][E];
    if (wk < ntiles) {
#pragma unroll
        for (int q = 0; q < 6; ++q) load_col<T, P>(v[q], make_rsrc(src + q * cs, cbytes), cur.voff, sstep);
    }
    while (wk < ntiles) {  // uniform over the workgroup
        if (MODE != Z_JUMP) {
#pragma unroll
            for (int q = 0; q < 6; q += NC) {
                // FP64: re-derive the lane indices per group so that LDS addresses are
                // recomputed (cheap ALU) instead of being kept live across all transforms;
                // FP32, issue-bound with registers to spare, keeps them (5% fewer VALU
                // instructions, the pass 2% faster at 256^3)
                int tq = t, cq = c;
                if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(tq), "+v"(cq));
                lds.c = cq;
                fft_stages_n<P, 0, false, kStagedTw, EIFP_FUSED_CT, NC>(
                    reinterpret_cast<cpx<T>(&)[NC][E]>(v[q]), tq, lds, s_tw);
                if (EIFP_FUSED_SB & 1) __builtin_amdgcn_sched_barrier(0);  // one group's temporaries live at a time
            }
        }

        const double bx = cur.col == 0 ? 0.0 : pp.nu[0] * (double)cur.col;  // packed column: Omega_x = 0 at 0 and Nx/2
        const double bo = omega(cur.o, n_outer, AXIS == 1 ? pp.nu[2] : pp.nu[1]);
        const double w = cur.col == 0 ? 1.0 : 2.0;
        const bool sum = want_inv && cur.active;
        // basic record along y: per-pencil sums, scaled once (the order of the sums is fixed)
        constexpr bool kPencil = (Q == INV_NPART && AXIS == 1);
        PencilSums ps;
#pragma unroll
        for (int i = 0; i < E; ++i) {
            // after a forward transform register i holds position m_last(i); loaded from the
            // anchored spectrum it holds m_first(i), which is also what the inverse expects
            const int kp = t + TT * (MODE == Z_JUMP ? m_first<P>(i) : m_last<P>(i));
            const double bp = omega(kp, NZ, AXIS == 1 ? pp.nu[1] : pp.nu[2]);
            const double by = AXIS == 1 ? bp : bo;
            const double bz = AXIS == 1 ? bo : bp;
            cpx<T> h[3] = {v[0][i], v[1][i], v[2][i]};
            cpx<T> e[3] = {v[3][i], v[4][i], v[5][i]};
            if (MODE == Z_STEP || MODE == Z_JUMP) {
                propagate_mode(h, e, bx, by, bz, pp);
            } else {
                const T s = (T)pp.inv_ns;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    h[q] = scale(h[q], s);
                    e[q] = scale(e[q], s);
                }
            }
            if (sum) {
                if constexpr (kPencil) ps.add(bx, by, bz, h, e);
                else accumulate_invariants<Q>(acc, w, bx, by, bz, h, e, pp);
            }
            if (MODE == Z_STEP || MODE == Z_JUMP) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    v[q][i] = h[q];
                    v[3 + q][i] = e[q];
                }
            }
            if (EIFP_FUSED_SB & 2) __builtin_amdgcn_sched_barrier(0);  // one mode's temporaries live at a time
        }
        if constexpr (kPencil) {
            if (sum) {
                double a[INV_NPART];
                ps.finish(a, w, bx, bo, pp);
#pragma unroll
                for (int q = 0; q < INV_NPART; ++q) acc[q] += a[q];
            }
        }

        ++k;
        const int wn = PERSIST ? persist_tile(k, G) : ntiles;
        const bool more = PERSIST && wn < ntiles;
        const Tile nxt = tile(more ? wn : wk);
        if (MODE == Z_STEP || MODE == Z_JUMP) {
            // inverse transform and store each component as soon as it is done, then
            // start loading the same component of the next tile into its registers
#pragma unroll
            for (int q = 0; q < 6; q += NC) {
#pragma unroll
                for (int n = 0; n < NC; ++n)
                    if (MODE == Z_STEP) last_to_first<P>(v[q + n]);
                int tq = t, cq = c;
                if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(tq), "+v"(cq));
                lds.c = cq;
                fft_stages_n<P, 0, true, kStagedTw, EIFP_FUSED_CT, NC>(
                    reinterpret_cast<cpx<T>(&)[NC][E]>(v[q]), tq, lds, s_tw);
                if (EIFP_FUSED_DRAIN && q + NC == 6) {
                    // last group: its stores, a wait until every outstanding vector memory
                    // operation has completed, then its next-tile loads, so that the wait
                    // for the next tile's data at the top of the loop covers loads only
#pragma unroll
                    for (int n = 0; n < NC; ++n)
                        store_col<T, P, EIFP_FUSED_ST_AUX>(v[q + n], make_rsrc(buf + (q + n) * cs, cbytes), cur.voff, sstep, cur.active);
                    if (more) {
                        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt not waited for
#pragma unroll
                        for (int n = 0; n < NC; ++n)
                            load_col<T, P>(v[q + n], make_rsrc(src + (q + n) * cs, cbytes), nxt.voff, sstep);
                    }
                } else {
#pragma unroll
                    for (int n = 0; n < NC; ++n) {
                        store_col<T, P, EIFP_FUSED_ST_AUX>(v[q + n], make_rsrc(buf + (q + n) * cs, cbytes), cur.voff, sstep, cur.active);
                        if (more) load_col<T, P>(v[q + n], make_rsrc(src + (q + n) * cs, cbytes), nxt.voff, sstep);
                    }
                }
                if (EIFP_FUSED_SB & 1) __builtin_amdgcn_sched_barrier(0);
            }
        } else if (more) {
            // Z_FORWARD leaves memory untouched
#pragma unroll
            for (int q = 0; q < 6; ++q) load_col<T, P>(v[q], make_rsrc(src + q * cs, cbytes), nxt.voff, sstep);
        }
        wk = wn;
        cur = nxt;
    }
    if (want_inv) block_reduce_store<NT, Q>(acc, mem.partials + (long)blockIdx.x * Q, s_red);
}

// ---------------------------------------------------------------------------------
// fused pass, split form: the tile is held by two thread groups of NG = T B threads;
// group 0 transforms the H components (0-2), group 1 the E components (3-5), so each
// thread holds 3 E values instead of 6 E and twice the waves fit in the register file.
// Between the transforms the two partners of a pencil position (same column and thread
// index t, one in each group, NG threads apart) trade halves through LDS: group 0 takes
// the modes of register slots [0, E/2) of all six components, group 1 the slots
// [E/2, E); each propagates its modes and accumulates their invariant sums, and the
// partners trade back before the inverse transforms.
// ---------------------------------------------------------------------------------
#ifndef EIFP_ZSWAVES64
#define EIFP_ZSWAVES64 2
#endif
#ifndef EIFP_ZSWAVES32
#define EIFP_ZSWAVES32 3
#endif
template <typename T, class P> struct ZWavesS {
    // 12 values per thread: one wave in FP64 (36 complex values held), two in FP32
    static constexpr int value = sizeof(T) == 8 ? (P::E >= 12 ? 1 : EIFP_ZSWAVES64)
                                                : (P::N % 3 == 0 ? 2 : EIFP_ZSWAVES32);
};

// swap area: [slot][thread] reals, slot-major so that consecutive threads use
// consecutive banks; a complex slot k occupies real slots 2k (re) and 2k + 1 (im)
template <typename T, int NT>
__device__ __forceinline__ void swap_put(T* sw, int slot, cpx<T> a) {
    sw[(2 * slot) * NT + threadIdx.x] = a.x;
    sw[(2 * slot + 1) * NT + threadIdx.x] = a.y;
}
template <typename T, int NT>
__device__ __forceinline__ cpx<T> swap_get(const T* sw, int slot, int from) {
    return {sw[(2 * slot) * NT + from], sw[(2 * slot + 1) * NT + from]};
}

// The work of one group (G = 0: H, 1: E) between the transforms; G is a template
// parameter so that every register index is a compile-time constant.  The callers
// branch on the group, which is uniform per wave, and keep every barrier outside.
template <typename T, class P, int MODE, int AXIS, int G, int NT>
struct SplitHalf {
    static constexpr int E = P::E, EH = E / 2, TT = P::T, NZ = P::N;
    static constexpr int KEEP = G * EH;       // register slots this group keeps
    static constexpr int SEND = EH - KEEP;    // and the ones it hands to its partner

    static __device__ __forceinline__ void put(const cpx<T> (&v)[3][E], T* sw) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int j = 0; j < EH; ++j) swap_put<T, NT>(sw, q * EH + j, v[q][SEND + j]);
    }

    // fetch the partner's components of the kept modes into o, propagate (or scale) the
    // kept modes of all six components, accumulate their invariant sums into acc
    template <int Q>
    static __device__ __forceinline__ void modes(cpx<T> (&v)[3][E], cpx<T> (&o)[3][EH], const T* sw, int partner,
                                                 int t, double bx, double bo, double w, bool sum,
                                                 const PropParams& pp, double (&acc)[Q]) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int j = 0; j < EH; ++j) o[q][j] = swap_get<T, NT>(sw, q * EH + j, partner);
        constexpr bool kPencil = (Q == INV_NPART && AXIS == 1);
        PencilSums ps;
#pragma unroll
        for (int j = 0; j < EH; ++j) {
            const int i = KEEP + j;
            const int kp = t + TT * (MODE == Z_JUMP ? m_first<P>(i) : m_last<P>(i));
            const double bp = omega(kp, NZ, AXIS == 1 ? pp.nu[1] : pp.nu[2]);
            const double by = AXIS == 1 ? bp : bo;
            const double bz = AXIS == 1 ? bo : bp;
            cpx<T> h[3], e[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                h[q] = G == 0 ? v[q][i] : o[q][j];
                e[q] = G == 0 ? o[q][j] : v[q][i];
            }
            if (MODE == Z_STEP || MODE == Z_JUMP) {
                propagate_mode(h, e, bx, by, bz, pp);
            } else {
                const T s = (T)pp.inv_ns;
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    h[q] = scale(h[q], s);
                    e[q] = scale(e[q], s);
                }
            }
            if (sum) {
                if constexpr (kPencil) ps.add(bx, by, bz, h, e);
                else accumulate_invariants<Q>(acc, w, bx, by, bz, h, e, pp);
            }
            if (MODE == Z_STEP || MODE == Z_JUMP) {
#pragma unroll
                for (int q = 0; q < 3; ++q) {
                    v[q][i] = G == 0 ? h[q] : e[q];
                    o[q][j] = G == 0 ? e[q] : h[q];
                }
            }
            if (EIFP_FUSED_SB & 2) __builtin_amdgcn_sched_barrier(0);
        }
        if constexpr (kPencil) {
            if (sum) {
                double a[INV_NPART];
                ps.finish(a, w, bx, bo, pp);
#pragma unroll
                for (int q = 0; q < INV_NPART; ++q) acc[q] += a[q];
            }
        }
    }

    // hand the partner's propagated components back, and take this group's
    static __device__ __forceinline__ void put_back(const cpx<T> (&o)[3][EH], T* sw) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int j = 0; j < EH; ++j) swap_put<T, NT>(sw, q * EH + j, o[q][j]);
    }
    static __device__ __forceinline__ void get_back(cpx<T> (&v)[3][E], const T* sw, int partner) {
#pragma unroll
        for (int q = 0; q < 3; ++q)
#pragma unroll
            for (int j = 0; j < EH; ++j) v[q][SEND + j] = swap_get<T, NT>(sw, q * EH + j, partner);
    }
};

// Same launch geometry, persistence and partial records as k_fused, with 2 T B threads
// per block; persistent workgroups (ZPersistS) load the next tile's components as the
// current tile's inverse transforms store theirs.
#ifndef EIFP_ZSPERSIST64
#define EIFP_ZSPERSIST64 1
#endif
#ifndef EIFP_ZSPERSIST32
#define EIFP_ZSPERSIST32 0
#endif
template <typename T, class P> struct ZPersistS {
    // FP64 at one wave per SIMD (12 values per thread) has the registers for it; at two
    // waves the loop state spills
    static constexpr bool value = sizeof(T) == 8 ? (EIFP_ZSPERSIST64 != 0 && P::E >= 12) : EIFP_ZSPERSIST32 != 0;
};

template <typename T, class P, int B, int MODE, int AXIS>
__global__ void __launch_bounds__(2 * P::T * B, (ZWavesS<T, P>::value))
k_fused_split(const MemberDesc<T>* __restrict__ md, int M, int n_outer, int ntx, long pstride, long ostride, long cs,
              const cpx<T>* __restrict__ tw, int want_inv) {
    constexpr bool PERSIST = ZPersistS<T, P>::value;
    constexpr int E = P::E, TT = P::T, NG = P::T * B, NT = 2 * NG, EH = E / 2;
    constexpr int PLANE = zplane<P, B>();
    static_assert(NG % 64 == 0, "each group must be whole waves");
    static_assert(E % 2 == 0, "the modes are split in halves");
    static_assert(3 * E * NT <= 8 * PLANE, "the swap area fits in the exchange buffers");
    __shared__ T s_x[8 * PLANE];  // per group: two exchange buffers (re, im); also the swap area
    __shared__ cpx<T> s_tw[P::N * TwParts<T>::value];
    constexpr int Q = NQ<MODE>::value;
    __shared__ double s_red[(NT / 64) * Q];
    stage_table_plan<P>(s_tw, tw);  // ordered by stage (conflict-free reads)
    const MemberDesc<T>& mem = md[blockIdx.z];
    const PropParams pp = mem.pp;
    cpx<T>* buf = mem.work;
    const int g = (int)threadIdx.x / NG;  // uniform per wave
    const int lt = (int)threadIdx.x - g * NG;
    const int c = lt % B, t = lt / B;
    const int partner = g ? (int)threadIdx.x - NG : (int)threadIdx.x + NG;
    const int G = (int)gridDim.x, ntiles = ntx * n_outer;
    const unsigned cbytes = (unsigned)cs * sizeof(cpx<T>);
    const unsigned sstep = (unsigned)(TT * pstride) * sizeof(cpx<T>);
    LdsCols2<T, B, PLANE, zcol_pitch(B), zskew<P>()> lds{s_x + g * 4 * PLANE, c, 0};
    cpx<T>* own = buf + 3 * g * cs;
    const cpx<T>* src = MODE == Z_JUMP ? mem.spec + 3 * g * cs : own;
    struct Tile {
        int col, o;
        bool active;
        unsigned voff;
    };
    auto tile = [&](int w) {
        Tile a;
        a.col = (w % ntx) * B + c;
        a.o = w / ntx;
        a.active = a.col < M;
        a.voff = (unsigned)(t * pstride + a.o * ostride + (a.active ? a.col : M - 1)) * sizeof(cpx<T>);
        return a;
    };
    using H0 = SplitHalf<T, P, MODE, AXIS, 0, NT>;
    using H1 = SplitHalf<T, P, MODE, AXIS, 1, NT>;

    double acc[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) acc[q] = 0.0;
    int k = 0;
    int wk = persist_tile(0, G);
    Tile cur = tile(wk < ntiles ? wk : 0);
    cpx<T> v[3][E];
    if (wk < ntiles) {
#pragma unroll
        for (int q = 0; q < 3; ++q) load_col<T, P>(v[q], make_rsrc(src + q * cs, cbytes), cur.voff, sstep);
    }
    while (wk < ntiles) {  // uniform over the workgroup
        if (MODE != Z_JUMP) {
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                int tq = t, cq = c;
                if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(tq), "+v"(cq));  // as in k_fused
                lds.c = cq;
                fft_pencil<P, false, kStagedTw, EIFP_FUSED_CT>(v[q], tq, lds, s_tw);
                if (EIFP_FUSED_SB & 1) __builtin_amdgcn_sched_barrier(0);
            }
        }
        const double bx = cur.col == 0 ? 0.0 : pp.nu[0] * (double)cur.col;  // packed column: Omega_x = 0 at 0 and Nx/2
        const double bo = omega(cur.o, n_outer, AXIS == 1 ? pp.nu[2] : pp.nu[1]);
        const double w = cur.col == 0 ? 1.0 : 2.0;
        const bool sum = want_inv && cur.active;
        cpx<T> oth[3][EH];
        __syncthreads();  // every exchange of the forward transforms has been read
        if (g == 0) H0::put(v, s_x);
        else H1::put(v, s_x);
        __syncthreads();
        if (g == 0) H0::template modes<Q>(v, oth, s_x, partner, t, bx, bo, w, sum, pp, acc);
        else H1::template modes<Q>(v, oth, s_x, partner, t, bx, bo, w, sum, pp, acc);
        __syncthreads();  // the swap area has been read
        ++k;
        const int wn = PERSIST ? persist_tile(k, G) : ntiles;
        const bool more = PERSIST && wn < ntiles;
        const Tile nxt = tile(more ? wn : wk);
        if (MODE == Z_STEP || MODE == Z_JUMP) {
            if (g == 0) H0::put_back(oth, s_x);
            else H1::put_back(oth, s_x);
            __syncthreads();
            if (g == 0) H0::get_back(v, s_x, partner);
            else H1::get_back(v, s_x, partner);
            __syncthreads();  // before the inverse transforms reuse the area as exchange buffers
#pragma unroll
            for (int q = 0; q < 3; ++q) {
                if (MODE == Z_STEP) last_to_first<P>(v[q]);
                int tq = t, cq = c;
                if constexpr (sizeof(T) == 8) asm volatile("" : "+v"(tq), "+v"(cq));  // as in k_fused
                lds.c = cq;
                fft_pencil<P, true, kStagedTw, EIFP_FUSED_CT>(v[q], tq, lds, s_tw);
                store_col<T, P, EIFP_FUSED_ST_AUX>(v[q], make_rsrc(own + q * cs, cbytes), cur.voff, sstep, cur.active);
                if (more) load_col<T, P>(v[q], make_rsrc(src + q * cs, cbytes), nxt.voff, sstep);
                if (EIFP_FUSED_SB & 1) __builtin_amdgcn_sched_barrier(0);
            }
        } else if (more) {
#pragma unroll
            for (int q = 0; q < 3; ++q) load_col<T, P>(v[q], make_rsrc(src + q * cs, cbytes), nxt.voff, sstep);
        }
        wk = wn;
        cur = nxt;
    }
    if (want_inv) block_reduce_store<NT, Q>(acc, mem.partials + (long)blockIdx.x * Q, s_red);
}

// Twiddle table of length n: tw[k] = exp(-2 pi i k / n) for k < n, formed in FP64 and
// rounded to T; an FP32 table also holds the rounding remainders (FP64 value minus the
// rounded value, rounded) at tw[n + k].  Every table the library uses comes from here.
template <typename T>
__device__ __forceinline__ void form_twiddle(cpx<T>* __restrict__ tw, int n, int k) {
    const double a = 6.283185307179586476925286766559 * (double)k / (double)n;
    double sn, cs;
    sincos(a, &sn, &cs);
    sn = -sn;
    const cpx<T> hi = {(T)cs, (T)sn};
    tw[k] = hi;
    if constexpr (TwParts<T>::value == 2) tw[n + k] = {(T)(cs - (double)hi.x), (T)(sn - (double)hi.y)};
}
template <typename T>
__global__ void __launch_bounds__(256) k_twiddles(cpx<T>* __restrict__ tw, int n) {
    const int k = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < n) form_twiddle(tw, n, k);
}

// FP64 <-> T conversion for upload / download of the state.
template <typename TO, typename TI>
__global__ void __launch_bounds__(256) k_convert(const TI* __restrict__ in, TO* __restrict__ out, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long stride = (long)gridDim.x * blockDim.x;
    for (long q = i; q < n; q += stride) out[q] = (TO)in[q];
}

}  // namespace eifp
