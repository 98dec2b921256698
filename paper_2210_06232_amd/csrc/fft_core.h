// fft_core.h -- register/LDS Stockham FFT building blocks for gfx950 (wave64).
//
// A pencil of length N is held by T = N/E threads, E complex values each.  Thread t
// always owns the positions t + T*m, m < E, both when it loads the pencil and when
// it stores the transform, so a tile of pencils is read and written with the same
// coalesced pattern.  Between radix stages the data are exchanged through LDS
// (Stockham autosort: every stage reads at stride N/R and writes in expanded order,
// so the output comes out in natural order with no bit reversal).
//
// Transforms are unnormalised: forward X[k] = sum_j x[j] exp(-2 pi i jk/N), inverse
// with exp(+2 pi i jk/N) -- the DFT matrix of Sec. 2.3 of Wang & Jiang and N times
// its inverse.
#pragma once
#include <hip/hip_runtime.h>

namespace eifp {

template <typename T>
struct alignas(2 * sizeof(T)) cpx {
    T x, y;
};

template <typename T> __device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> __device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
// a b + c in one rounding.  Sums of two products below are written with it explicitly:
// under contraction the compiler would pick which of the two products to round first,
// and could pick differently in different kernels, so that the same transform written
// in two kernels (the x inverse and forward, alone and combined) would differ in the
// last bit.
__device__ __forceinline__ double fmat(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmat(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
template <typename T> __device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
    return {fmat(a.x, b.x, -(a.y * b.y)), fmat(a.x, b.y, a.y * b.x)};
}
// a * conj(b)
template <typename T> __device__ __forceinline__ cpx<T> cmulc(cpx<T> a, cpx<T> b) {
    return {fmat(a.x, b.x, a.y * b.y), fmat(a.y, b.x, -(a.x * b.y))};
}
template <typename T> __device__ __forceinline__ cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }

// Twiddle tables hold exp(-2 pi i k / n), k < n, formed in FP64.  In FP32 the rounded
// values are biased in modulus (sqrt(2)/2, for one, rounds down and enters every
// stage), so every transform would lose about one unit roundoff of energy and the
// error of a long FP32 run would grow linearly.  FP32 tables therefore carry a second
// part, lo = (FP64 value - hi) rounded, at index k + n, and every FP32 twiddle product
// adds the lo terms inside its FMA chain, before the single final rounding.
template <typename T> struct TwParts { static constexpr int value = 1; };
template <> struct TwParts<float> { static constexpr int value = 2; };

// v * w or v * conj(w) for the table entry k of a table of n entries (lo part at k + n;
// CT = false uses the rounded value alone)
template <bool CONJ, bool CT = true, typename T>
__device__ __forceinline__ cpx<T> twmul(const cpx<T>* tw, int k, int n, cpx<T> v) {
    const cpx<T> h = tw[k];
    if constexpr (TwParts<T>::value == 1 || !CT) {
        return CONJ ? cmulc(v, h) : cmul(v, h);
    } else {
        const cpx<T> l = tw[k + n];
        if (CONJ)
            return {__builtin_fmaf(v.x, h.x, __builtin_fmaf(v.y, h.y, __builtin_fmaf(v.x, l.x, v.y * l.y))),
                    __builtin_fmaf(v.y, h.x, __builtin_fmaf(-v.x, h.y, __builtin_fmaf(v.y, l.x, -(v.x * l.y))))};
        return {__builtin_fmaf(v.x, h.x, __builtin_fmaf(-v.y, h.y, __builtin_fmaf(v.x, l.x, -(v.y * l.y)))),
                __builtin_fmaf(v.x, h.y, __builtin_fmaf(v.y, h.x, __builtin_fmaf(v.x, l.y, v.y * l.x)))};
    }
}

// v * (c + i s) for FP64 constants c, s: in FP32 with the same two-part compensation
template <typename T>
__device__ __forceinline__ cpx<T> rotc(double c, double s, cpx<T> v) {
    if constexpr (sizeof(T) == 8) {
        return {fmat(v.x, c, -(v.y * s)), fmat(v.x, s, v.y * c)};
    } else {
        const float ch = (float)c, sh = (float)s;
        const float cl = (float)(c - (double)ch), sl = (float)(s - (double)sh);
        return {__builtin_fmaf(v.x, ch, __builtin_fmaf(-v.y, sh, __builtin_fmaf(v.x, cl, -(v.y * sl)))),
                __builtin_fmaf(v.x, sh, __builtin_fmaf(v.y, ch, __builtin_fmaf(v.x, sl, v.y * cl)))};
    }
}

// a * c for an FP64 constant c, compensated in FP32
template <typename T>
__device__ __forceinline__ T mulc(double c, T a) {
    if constexpr (sizeof(T) == 8) {
        return a * c;
    } else {
        const float ch = (float)c, cl = (float)(c - (double)ch);
        return __builtin_fmaf(a, ch, a * cl);
    }
}
template <typename T> __device__ __forceinline__ cpx<T> scale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
// multiply by i and by -i
template <typename T> __device__ __forceinline__ cpx<T> muli(cpx<T> a) { return {-a.y, a.x}; }
template <typename T> __device__ __forceinline__ cpx<T> mulmi(cpx<T> a) { return {a.y, -a.x}; }

// cos(2 pi j / 48) for j = 0..12, correctly rounded; every in-register twiddle
// exp(-+2 pi i e / R) with R | 48 is read off this quarter period.
constexpr double kCos48q[13] = {
    1.0, 0.9914448613738104, 0.9659258262890683, 0.9238795325112867,
    0.8660254037844386, 0.7933533402912352, 0.7071067811865476, 0.6087614290087207,
    0.5, 0.3826834323650898, 0.25881904510252074, 0.1305261922200516, 0.0};

__host__ __device__ constexpr double cos48(int j) {
    // j in [0, 48)
    return j <= 12 ? kCos48q[j] : j <= 24 ? -kCos48q[24 - j] : j <= 36 ? -kCos48q[j - 24] : kCos48q[48 - j];
}
__host__ __device__ constexpr double sin48(int j) { return cos48((j + 36) % 48); }

// v * exp(s 2 pi i e / R), s = -1 forward, +1 inverse; e and R are compile-time after
// unrolling, so the branches fold and +-1, +-i cost no arithmetic.
template <int R, bool INV, typename T>
__device__ __forceinline__ cpx<T> twc(int e, cpx<T> v) {
    e %= R;
    if (e == 0) return v;
    if ((4 * e) % R == 0) {
        const int q = 4 * e / R;  // quarter turns
        if (q == 2) return {-v.x, -v.y};
        const bool plus_i = (q == 1) == INV;  // forward: q=1 -> -i
        return plus_i ? muli(v) : mulmi(v);
    }
    const int j = (48 / R) * e;
    return rotc<T>(cos48(j), INV ? sin48(j) : -sin48(j), v);
}

// ---------------------------------------------------------------------------------
// small DFTs in registers
// ---------------------------------------------------------------------------------
template <int R, bool INV, typename T> struct Dft;

template <bool INV, typename T> struct Dft<1, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>*) {}
};

template <bool INV, typename T> struct Dft<2, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) {
        const cpx<T> t = a[0];
        a[0] = t + a[1];
        a[1] = t - a[1];
    }
};

template <bool INV, typename T> struct Dft<3, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) {
        // w = exp(-+2 pi i/3) = -1/2 -+ i sqrt(3)/2
        constexpr double h = 0.8660254037844386;
        const cpx<T> s = a[1] + a[2];
        const cpx<T> d = a[1] - a[2];
        const cpx<T> m = {a[0].x - (T)0.5 * s.x, a[0].y - (T)0.5 * s.y};
        // i * sin * d with sin = -+sqrt(3)/2
        const T hy = mulc<T>(h, d.y), hx = mulc<T>(h, d.x);
        const cpx<T> r = INV ? cpx<T>{-hy, hx} : cpx<T>{hy, -hx};
        a[0] = a[0] + s;
        a[1] = m + r;
        a[2] = m - r;
    }
};

template <bool INV, typename T> struct Dft<4, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) {
        const cpx<T> t0 = a[0] + a[2], t1 = a[0] - a[2];
        const cpx<T> t2 = a[1] + a[3], t3 = a[1] - a[3];
        const cpx<T> r = INV ? muli(t3) : mulmi(t3);
        a[0] = t0 + t2;
        a[2] = t0 - t2;
        a[1] = t1 + r;
        a[3] = t1 - r;
    }
};

// Cooley-Tukey split R = R1 R2 in registers:
//   X[k1 + R1 k2] = sum_n2 W_R2^{n2 k2} W_R^{n2 k1} sum_n1 x[R2 n1 + n2] W_R1^{n1 k1}
template <int R1, int R2, bool INV, typename T>
__device__ __forceinline__ void dft_split(cpx<T>* a) {
    constexpr int R = R1 * R2;
    cpx<T> y[R];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        cpx<T> t[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) t[n1] = a[R2 * n1 + n2];
        Dft<R1, INV, T>::run(t);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) y[n2 * R1 + k1] = twc<R, INV>(n2 * k1, t[k1]);
    }
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        cpx<T> t[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) t[n2] = y[n2 * R1 + k1];
        Dft<R2, INV, T>::run(t);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) a[k1 + R1 * k2] = t[k2];
    }
}

template <bool INV, typename T> struct Dft<6, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) { dft_split<3, 2, INV, T>(a); }
};
template <bool INV, typename T> struct Dft<8, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) { dft_split<4, 2, INV, T>(a); }
};
template <bool INV, typename T> struct Dft<12, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) { dft_split<4, 3, INV, T>(a); }
};
template <bool INV, typename T> struct Dft<16, INV, T> {
    __device__ __forceinline__ static void run(cpx<T>* a) { dft_split<4, 4, INV, T>(a); }
};

// ---------------------------------------------------------------------------------
// plans: N = product of the stage radices, each radix divides E (values per thread)
// ---------------------------------------------------------------------------------
template <int N_, int E_, int... Rs>
struct PlanDef {
    static constexpr int N = N_, E = E_, T = N_ / E_, S = sizeof...(Rs);
    static constexpr int R[S] = {Rs...};
};

template <int N, int E> struct Plan;
#define EIFP_PLAN(N, E, ...) \
    template <> struct Plan<N, E> : PlanDef<N, E, __VA_ARGS__> {};
EIFP_PLAN(2, 2, 2)
EIFP_PLAN(3, 3, 3)
EIFP_PLAN(4, 4, 4)
EIFP_PLAN(6, 6, 6)
EIFP_PLAN(8, 8, 8)
EIFP_PLAN(12, 12, 12)
EIFP_PLAN(12, 6, 6, 2)
EIFP_PLAN(16, 16, 16)
EIFP_PLAN(16, 8, 8, 2)
EIFP_PLAN(16, 4, 4, 4)
EIFP_PLAN(24, 12, 12, 2)
EIFP_PLAN(24, 6, 6, 2, 2)
EIFP_PLAN(32, 16, 16, 2)
EIFP_PLAN(32, 8, 8, 4)
EIFP_PLAN(48, 12, 12, 4)
EIFP_PLAN(48, 6, 6, 2, 2, 2)
EIFP_PLAN(64, 16, 16, 4)
EIFP_PLAN(64, 8, 8, 8)
EIFP_PLAN(96, 12, 12, 4, 2)
EIFP_PLAN(96, 6, 6, 2, 2, 2, 2)
EIFP_PLAN(128, 16, 16, 8)
EIFP_PLAN(128, 8, 8, 8, 2)
EIFP_PLAN(192, 12, 12, 4, 4)
EIFP_PLAN(256, 16, 16, 16)
EIFP_PLAN(256, 8, 8, 8, 4)
EIFP_PLAN(384, 12, 12, 4, 4, 2)
EIFP_PLAN(512, 16, 16, 16, 2)
EIFP_PLAN(512, 8, 8, 8, 8)
// four and six values per thread (low register pressure, for the six-component z pass in FP64)
EIFP_PLAN(8, 4, 4, 2)
EIFP_PLAN(32, 4, 4, 4, 2)
EIFP_PLAN(64, 4, 4, 4, 4)
EIFP_PLAN(128, 4, 4, 4, 4, 2)
EIFP_PLAN(256, 4, 4, 4, 4, 4)
EIFP_PLAN(512, 4, 4, 4, 4, 4, 2)
EIFP_PLAN(192, 6, 6, 2, 2, 2, 2, 2)
EIFP_PLAN(384, 6, 6, 2, 2, 2, 2, 2, 2)
#undef EIFP_PLAN

template <class P, int s>
__host__ __device__ constexpr int span_before() {  // product of the radices of stages < s
    int p = 1;
    for (int i = 0; i < s; ++i) p *= P::R[i];
    return p;
}

// Register index idx of the first stage (idx = u R0 + r) owns position t + T*m0(idx);
// after the last stage, idx = u RL + r owns position t + T*mL(idx).
template <class P>
__host__ __device__ constexpr int m_first(int idx) {
    return idx / P::R[0] + (idx % P::R[0]) * (P::E / P::R[0]);
}
template <class P>
__host__ __device__ constexpr int m_last(int idx) {
    return idx / P::R[P::S - 1] + (idx % P::R[P::S - 1]) * (P::E / P::R[P::S - 1]);
}

// Runs stages s..S-1.  v holds stage-s inputs: v[u R + r] = x[j + r N/R], j = t + T u.
// tw[k * TWS] = exp(-2 pi i k / N) for k < N (forward table; conj for the inverse).
// Lds provides st(pos, v), ld(pos) for this thread's pencil and sync().
// Stage twiddles come from tw[k * TWS] = exp(-2 pi i k / N), or, with TWS = kStagedTw,
// from a table in the plan's stage order (stage_table_plan), where the R - 1 factors of
// stage s for butterfly j are entries (NS - R_0) + (r - 1) NS + j mod NS: the lanes of one
// read then take consecutive entries instead of entries a power of two apart.
constexpr int kStagedTw = 0;
// CT: bit s set = the twiddle products of stage s use the table's lo parts (FP32 only)
constexpr int kCompAll = -1;
template <class P, int s, bool INV, int TWS, int CT = kCompAll, typename T, class Lds>
__device__ __forceinline__ void fft_stages(cpx<T> (&v)[P::E], int t, Lds& lds, const cpx<T>* __restrict__ tw) {
    constexpr int N = P::N, E = P::E, TT = P::T;
    constexpr int R = P::R[s];
    constexpr int NS = span_before<P, s>();
    constexpr int NB = E / R;
#pragma unroll
    for (int u = 0; u < NB; ++u) {
        const int j = t + TT * u;
        if constexpr (NS > 1) {
            const int jm = j % NS;
#pragma unroll
            for (int r = 1; r < R; ++r) {
                if constexpr (TWS == kStagedTw)
                    v[u * R + r] = twmul<INV, ((CT >> s) & 1) != 0>(tw, (NS - P::R[0]) + (r - 1) * NS + jm, N, v[u * R + r]);
                else
                    v[u * R + r] = twmul<INV, ((CT >> s) & 1) != 0>(tw, (jm * r * (N / (NS * R))) * TWS, N * TWS, v[u * R + r]);
            }
        }
        Dft<R, INV, T>::run(&v[u * R]);
    }
    if constexpr (s + 1 < P::S) {
        constexpr int R2 = P::R[s + 1];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = t + TT * u;
            const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
            for (int r = 0; r < R; ++r) lds.st(base + r * NS, v[u * R + r]);
        }
        lds.sync();
#pragma unroll
        for (int u = 0; u < E / R2; ++u) {
            const int j = t + TT * u;
#pragma unroll
            for (int r = 0; r < R2; ++r) v[u * R2 + r] = lds.ld(j + r * (N / R2));
        }
        lds.after_load();
        fft_stages<P, s + 1, INV, TWS, CT>(v, t, lds, tw);
    }
}

// After a forward transform the registers are in last-stage order; an inverse
// transform expects first-stage order.  Permute in registers (compile-time indices).
template <class P>
__host__ __device__ constexpr int last_slot_of_first(int idx) {
    // the idx' with m_last(idx') == m_first(idx)
    int found = 0;
    for (int k = 0; k < P::E; ++k)
        if (m_last<P>(k) == m_first<P>(idx)) found = k;
    return found;
}

template <class P, typename T>
__device__ __forceinline__ void last_to_first(cpx<T> (&v)[P::E]) {
    cpx<T> w[P::E];
#pragma unroll
    for (int i = 0; i < P::E; ++i) w[i] = v[last_slot_of_first<P>(i)];
#pragma unroll
    for (int i = 0; i < P::E; ++i) v[i] = w[i];
}

// NC pencils of the same thread transformed in lockstep: every exchange moves all NC
// through LDS behind one synchronisation (Lds::st / ld take the pencil index), so the NC
// transforms share their barriers and give the scheduler NC independent butterflies.
template <class P, int s, bool INV, int TWS, int CT, int NC, typename T, class Lds>
__device__ __forceinline__ void fft_stages_n(cpx<T> (&v)[NC][P::E], int t, Lds& lds, const cpx<T>* __restrict__ tw) {
    constexpr int N = P::N, E = P::E, TT = P::T;
    constexpr int R = P::R[s];
    constexpr int NS = span_before<P, s>();
    constexpr int NB = E / R;
#pragma unroll
    for (int n = 0; n < NC; ++n) {
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int j = t + TT * u;
            if constexpr (NS > 1) {
                const int jm = j % NS;
#pragma unroll
                for (int r = 1; r < R; ++r) {
                    if constexpr (TWS == kStagedTw)
                        v[n][u * R + r] = twmul<INV, ((CT >> s) & 1) != 0>(tw, (NS - P::R[0]) + (r - 1) * NS + jm, N, v[n][u * R + r]);
                    else
                        v[n][u * R + r] = twmul<INV, ((CT >> s) & 1) != 0>(tw, (jm * r * (N / (NS * R))) * TWS, N * TWS, v[n][u * R + r]);
                }
            }
            Dft<R, INV, T>::run(&v[n][u * R]);
        }
    }
    if constexpr (s + 1 < P::S) {
        constexpr int R2 = P::R[s + 1];
#pragma unroll
        for (int n = 0; n < NC; ++n)
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int j = t + TT * u;
                const int base = (j / NS) * NS * R + (j % NS);
#pragma unroll
                for (int r = 0; r < R; ++r) lds.st(n, base + r * NS, v[n][u * R + r]);
            }
        lds.sync();
#pragma unroll
        for (int n = 0; n < NC; ++n)
#pragma unroll
            for (int u = 0; u < E / R2; ++u) {
                const int j = t + TT * u;
#pragma unroll
                for (int r = 0; r < R2; ++r) v[n][u * R2 + r] = lds.ld(n, j + r * (N / R2));
            }
        lds.after_load();
        fft_stages_n<P, s + 1, INV, TWS, CT, NC>(v, t, lds, tw);
    }
}

template <class P, bool INV, int TWS, int CT = kCompAll, typename T, class Lds>
__device__ __forceinline__ void fft_pencil(cpx<T> (&v)[P::E], int t, Lds& lds, const cpx<T>* __restrict__ tw) {
    fft_stages<P, 0, INV, TWS, CT>(v, t, lds, tw);
}

// LDS views.  Columns: a tile of B pencils stored [pos][col] (real and imaginary parts
// in separate planes), so the B lanes of one position hit consecutive banks.
// Rows of the [pos][col] views have a pitch of B + pad elements: positions that differ
// by a power of two then fall in different LDS banks (a pitch of B would put the lanes of
// a wave that share a column on the same banks).
#ifndef EIFP_LDS_PAD
#define EIFP_LDS_PAD 1
#endif
__host__ __device__ constexpr int col_pitch(int B) { return B + EIFP_LDS_PAD; }
// pad of the fused pass's exchange buffers (its narrow tiles measure best unpadded)
#ifndef EIFP_ZPAD
#define EIFP_ZPAD 0
#endif
__host__ __device__ constexpr int zcol_pitch(int B) { return B + EIFP_ZPAD; }
// rows of a [pos][col] buffer with one empty row after every 2^SK positions (SK > 0)
template <int N, int SK>
__host__ __device__ constexpr int skew_rows() { return N + (SK > 0 ? (N >> SK) + 1 : 0); }
// skew of the fused pass's exchange rows (see LdsCols2): power-of-two lengths and
// lengths with a factor 3
#ifndef EIFP_ZSKEW
#define EIFP_ZSKEW 1
#endif
#ifndef EIFP_ZSKEW3
#define EIFP_ZSKEW3 0
#endif
// (EIFP_ZSKEW = 1 selects log2 of the plan's first radix: the stage-0 writes of one
// register are that radix apart)
template <class P>
__host__ __device__ constexpr int zskew() {
    if (P::N % 3 == 0) return EIFP_ZSKEW3;
    if (EIFP_ZSKEW != 1) return EIFP_ZSKEW;
    int k = 0;
    while ((1 << k) < P::R[0]) ++k;
    return k;
}
template <class P, int B>
__host__ __device__ constexpr int zplane() { return skew_rows<P::N, zskew<P>()>() * zcol_pitch(B); }
// after_load(): a single buffer needs a second barrier before it is written again; the
// double-buffered views flip to the other buffer instead, which is safe because the
// next write to this buffer comes after the next exchange's barrier.
template <typename T, int B, int PITCH = col_pitch(B), int SK = 0>
struct LdsCols {
    T* re;
    T* im;
    int c;
    static __device__ __forceinline__ int at(int pos) { return (SK > 0 ? pos + (pos >> SK) : pos) * PITCH; }
    __device__ __forceinline__ void st(int pos, cpx<T> a) { re[at(pos) + c] = a.x; im[at(pos) + c] = a.y; }
    __device__ __forceinline__ cpx<T> ld(int pos) const { return {re[at(pos) + c], im[at(pos) + c]}; }
    __device__ __forceinline__ void sync() { __syncthreads(); }
    __device__ __forceinline__ void after_load() { __syncthreads(); }
};

// Two alternating [pos][col] buffers of PLANE reals per plane (re, im): one barrier per
// exchange.  base holds re0, im0, re1, im1.  With SK > 0 one empty row follows every 2^SK
// positions (row pos + (pos >> SK)): the stage-0 writes, whose positions are 8 apart for
// a fixed register, then fall in different banks, and the offsets between a thread's
// accesses stay compile-time constants.
template <typename T, int B, int PLANE, int PITCH = col_pitch(B), int SK = 0>
struct LdsCols2 {
    T* base;
    int c;
    int cur;
    static __device__ __forceinline__ int row(int pos) { return SK > 0 ? pos + (pos >> SK) : pos; }
    __device__ __forceinline__ T* re() const { return base + (2 * cur) * PLANE; }
    __device__ __forceinline__ void st(int pos, cpx<T> a) {
        T* r = re();
        r[row(pos) * PITCH + c] = a.x;
        r[PLANE + row(pos) * PITCH + c] = a.y;
    }
    __device__ __forceinline__ cpx<T> ld(int pos) const {
        const T* r = re();
        return {r[row(pos) * PITCH + c], r[PLANE + row(pos) * PITCH + c]};
    }
    __device__ __forceinline__ void sync() { __syncthreads(); }
    __device__ __forceinline__ void after_load() { cur ^= 1; }
};

// NC pencil sets in two alternating buffers: [buffer][set][re, im][PLANE reals], rows
// skewed as in LdsCols2; one barrier per exchange.
template <typename T, int B, int PLANE, int PITCH, int SK, int NC>
struct LdsColsN {
    T* base;
    int c;
    int cur;
    static __device__ __forceinline__ int row(int pos) { return SK > 0 ? pos + (pos >> SK) : pos; }
    __device__ __forceinline__ T* re(int n) const { return base + (2 * (cur * NC + n)) * PLANE; }
    __device__ __forceinline__ void st(int n, int pos, cpx<T> a) {
        T* r = re(n);
        r[row(pos) * PITCH + c] = a.x;
        r[PLANE + row(pos) * PITCH + c] = a.y;
    }
    __device__ __forceinline__ cpx<T> ld(int n, int pos) const {
        const T* r = re(n);
        return {r[row(pos) * PITCH + c], r[PLANE + row(pos) * PITCH + c]};
    }
    __device__ __forceinline__ void sync() { __syncthreads(); }
    __device__ __forceinline__ void after_load() { cur ^= 1; }
};

// Rows: P pencils stored one after another with pitch LD (at least rows_pitch<T>(M)),
// with one pad element after every 2^skew positions, so that positions a power of two
// apart (the stride of the first exchange) spread over the banks.  Measured best: every
// 8 in FP64, every 16 in FP32.
#ifndef EIFP_XSKEW64
#define EIFP_XSKEW64 3
#endif
#ifndef EIFP_XSKEW32
#define EIFP_XSKEW32 4
#endif
template <typename T> struct RowSkew { static constexpr int value = sizeof(T) == 8 ? EIFP_XSKEW64 : EIFP_XSKEW32; };
template <typename T>
__host__ __device__ constexpr int rows_pitch(int m) { return m + 1 + (RowSkew<T>::value ? m >> RowSkew<T>::value : 0); }
// Ordering of LDS traffic that stays within one wave: a wave's LDS instructions are
// performed in issue order, so a later read sees an earlier write of any lane of the
// same wave once the compiler keeps them in program order (wavefront-scope fences and a
// wave barrier; no instruction, no wait on other waves).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// A row's T threads are consecutive and T divides 64, so each row lies within one wave
// and its exchanges need only wave-scope ordering: the waves of a workgroup run their
// rows independently.
template <typename T, int LD>
struct LdsRows {
    T* re;
    T* im;
    int p;
    static __device__ __forceinline__ int at(int pos) {
        constexpr int sk = RowSkew<T>::value;
        return sk ? pos + (pos >> sk) : pos;
    }
    __device__ __forceinline__ void st(int pos, cpx<T> a) { re[p * LD + at(pos)] = a.x; im[p * LD + at(pos)] = a.y; }
    __device__ __forceinline__ cpx<T> ld(int pos) const { return {re[p * LD + at(pos)], im[p * LD + at(pos)]}; }
    __device__ __forceinline__ void sync() { wave_lds_sync(); }
    __device__ __forceinline__ void after_load() { wave_lds_sync(); }
};

// Copy a twiddle table of n entries into LDS (all threads of the block take part).
// Where the first FFT stage ends in a block barrier, no barrier is needed between this
// copy and the first read; the row kernels, whose exchanges are wave-local, place one
// after the copy.
template <typename T>
__device__ __forceinline__ void stage_table(cpx<T>* dst, const cpx<T>* __restrict__ src, int n) {
    // n entries, plus their lo parts for FP32 tables
    for (int i = threadIdx.x; i < n * TwParts<T>::value; i += blockDim.x) dst[i] = src[i];
}

// The stage-ordered table of plan P (N - 1 entries, then their lo parts at +N for FP32)
// from the plain table src[k] = exp(-2 pi i k / N); the caller synchronises before use.
template <class P, int s = 1, typename T>
__device__ __forceinline__ void stage_table_plan(cpx<T>* dst, const cpx<T>* __restrict__ src) {
    if constexpr (s < P::S) {
        constexpr int N = P::N, R = P::R[s], NS = span_before<P, s>(), off = NS - P::R[0];
        for (int i = threadIdx.x; i < NS * (R - 1); i += blockDim.x) {
            const int r = i / NS + 1, jm = i % NS;
            const int k = jm * r * (N / (NS * R));
            dst[off + i] = src[k];
            if constexpr (TwParts<T>::value == 2) dst[N + off + i] = src[N + k];
        }
        stage_table_plan<P, s + 1>(dst, src);
    }
}

// Raw buffer access (gfx9 descriptor): one SGPR descriptor per array, a per-lane VGPR
// byte offset and a wave-uniform SGPR byte offset.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T> struct BufIO;
template <> struct BufIO<double> {
    __device__ __forceinline__ static cpx<double> ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b128(r, (int)vo, (int)so, 0);
        return __builtin_bit_cast(cpx<double>, u);
    }
    template <int AUX = 0>
    __device__ __forceinline__ static void st(cpx<double> v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        using U4 = __attribute__((ext_vector_type(4))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v), r, (int)vo, (int)so, AUX);
    }
};
template <> struct BufIO<float> {
    __device__ __forceinline__ static cpx<float> ld(__amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        const auto u = __builtin_amdgcn_raw_buffer_load_b64(r, (int)vo, (int)so, 0);
        return __builtin_bit_cast(cpx<float>, u);
    }
    template <int AUX = 0>
    __device__ __forceinline__ static void st(cpx<float> v, __amdgpu_buffer_rsrc_t r, unsigned vo, unsigned so) {
        using U2 = __attribute__((ext_vector_type(2))) unsigned int;
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U2, v), r, (int)vo, (int)so, AUX);
    }
};

}  // namespace eifp
