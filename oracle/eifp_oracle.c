/*
 * eifp_oracle.c -- TEST INFRASTRUCTURE, NOT PRODUCT CODE.
 *
 * A plain, slow, obviously-correct FP64 CPU reference for the time-exponential-
 * integrator Fourier pseudospectral scheme of B. Wang and Y. L. Jiang,
 * "Time exponential integrator Fourier pseudospectral methods with high accuracy
 * and multiple conservation laws for three-dimensional Maxwell's equations"
 * (arXiv:2210.06232).
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header, table or helper with the
 * GPU library, and it includes nothing but libc / libm.
 *
 * What is here, and the passage each function follows:
 *   orc_dft          O(n^2) DFT with the matrix F_N(j,k) = exp(-2 pi i jk/N)   (Sec. 2.3)
 *   orc_fft          own mixed-radix FFT (recursive decimation in time)       (Sec. 2.3, Alg. 1 step 4)
 *   orc_wavenumbers  diagonal of Omega_w, Nyquist entry set to 0              (Sec. 2.3, Alg. 2 step 1)
 *   orc_dmatrix      cot-form spectral differentiation matrix D_w             (Sec. 2.2)
 *   orc_deriv        D_w applied along one axis via F^{-1} (i Omega_w) F      (Sec. 2.3)
 *   orc_fft3         F_{Nz} (x) F_{Ny} (x) F_{Nx} on an [nz][ny][nx] array    (Def. 2.3 step 2, Alg. 1)
 *   orc_coefficients c_ij, s_ij of Prop. 2.2 for one wavevector              (Prop. 2.2, Alg. 2 step 3)
 *   orc_propagator   the 6x6 block of exp(t Lambda-hat) for one wavevector    (Prop. 2.1/2.2, Alg. 2 step 4)
 *   orc_step         Algorithm 2, repeated nsteps times with dt = tau         (Def. 2.3, Alg. 2)
 *   orc_invariants   discrete energies, helicities, momenta, divergences in
 *                    physical space                                          (Thms 4.1, 4.3, 4.4, 4.6)
 *   orc_symplectic   bilinear form <E_U,H_V>_N - <E_V,H_U>_N between two
 *                    states (the quantity behind Thm 4.5)                     (Thm 4.5)
 *   orc_drift_scales Cauchy-Schwarz bounds of H1, M1_k and the divergence
 *                    norms, the scales their drift is measured against       (Thms 4.3, 4.4, 4.6)
 *
 * Readings where the paper is silent or garbled (each one listed in the design notes):
 *   - Psi = 0 (the zero mode, or a mode whose only nonzero index is a Nyquist index):
 *     r1 and r2 take their limits -1/2 and 1, so the mode is held fixed.
 *   - cosh(sqrt(-Psi)) and sinh(sqrt(-Psi))/sqrt(-Psi) with Psi >= 0 are cos(theta)
 *     and sin(theta)/theta with theta = sqrt(Psi).
 *   - the Nyquist entry of a_w is 0, as in the definition of Lambda_w (Sec. 2.3);
 *     the listing of Alg. 2 step 1 drops a minus sign on the next entry.
 *   - the discrete inner product is the grid mean (1/(Nx Ny Nz)) sum u v.
 *
 * Field layout: component-major [3][nz][ny][nx] doubles, x fastest (Sec. 2.2 vector
 * ordering, index Nx Ny (l-1) + Nx (k-1) + j).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

static const double ORC_PI = 3.14159265358979323846264338327950288;

/* ------------------------------------------------------------------------- */
/* 1-D transforms                                                             */
/* ------------------------------------------------------------------------- */

/* exp(sign * 2 pi i * j / n) with j reduced mod n first, so large products stay accurate. */
static cplx root_of_unity(long j, long n, int sign)
{
    long r = j % n;
    if (r < 0) r += n;
    double a = 2.0 * ORC_PI * (double)r / (double)n;
    return cos(a) + (double)sign * sin(a) * I;
}

/* Textbook O(n^2) DFT: out[k] = sum_j in[j] exp(sign 2 pi i jk/n).  sign = -1 is F_N
 * of Sec. 2.3; sign = +1 is n * F_N^{-1}.  Arrays are interleaved (re, im). */
int orc_dft(int n, const double *in, double *out, int sign)
{
    if (n <= 0 || (sign != 1 && sign != -1)) return 1;
    const cplx *x = (const cplx *)in;
    cplx *X = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!X) return 2;
    for (int k = 0; k < n; ++k) {
        cplx s = 0;
        for (int j = 0; j < n; ++j) s += x[j] * root_of_unity((long)j * k, n, sign);
        X[k] = s;
    }
    memcpy(out, X, sizeof(cplx) * (size_t)n);
    free(X);
    return 0;
}

static int smallest_factor(int n)
{
    for (int p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* Decimation in time.  With p the smallest factor of n and m = n/p, split x into the
 * p subsequences x[r + p s] (s < m), transform each (length m) into Y_r, and combine:
 *     X[k] = sum_{r<p} W^{r k} Y_r[k mod m],   W = exp(sign 2 pi i / n).
 * w[] holds W^j for j < n (the table of the top-level length; a sub-length n/q uses
 * every q-th entry, which is the same root of unity). */
static void fft_rec(int n, const cplx *x, long stride, cplx *X, int sign,
                    const cplx *w, long wstep, cplx *scratch)
{
    if (n == 1) { X[0] = x[0]; return; }
    int p = smallest_factor(n);
    int m = n / p;
    for (int r = 0; r < p; ++r)
        fft_rec(m, x + r * stride, stride * p, X + (long)r * m, sign, w, wstep * p, scratch);
    /* combine: X[k] for all k < n from Y_r = X[r m .. r m + m - 1] */
    for (int k = 0; k < n; ++k) {
        cplx s = 0;
        for (int r = 0; r < p; ++r) {
            long e = ((long)r * k) % n;               /* exponent of W (mod n) */
            s += w[e * wstep] * X[(long)r * m + (k % m)];
        }
        scratch[k] = s;
    }
    memcpy(X, scratch, sizeof(cplx) * (size_t)n);
}

/* Unnormalised transform of length n: out[k] = sum_j in[j] exp(sign 2 pi i jk/n). */
int orc_fft(int n, const double *in, double *out, int sign)
{
    if (n <= 0 || (sign != 1 && sign != -1)) return 1;
    cplx *w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *buf = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *scr = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    cplx *src = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!w || !buf || !scr || !src) { free(w); free(buf); free(scr); free(src); return 2; }
    for (int j = 0; j < n; ++j) w[j] = root_of_unity(j, n, sign);
    memcpy(src, in, sizeof(cplx) * (size_t)n);
    fft_rec(n, src, 1, buf, sign, w, 1, scr);
    memcpy(out, buf, sizeof(cplx) * (size_t)n);
    free(w); free(buf); free(scr); free(src);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* 3-D transform on an [nz][ny][nx] complex array                             */
/* ------------------------------------------------------------------------- */

typedef struct { int n; cplx *w, *buf, *scr, *src; } fft_plan;

static int plan_make(fft_plan *p, int n, int sign)
{
    p->n = n;
    p->w = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    p->buf = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    p->scr = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    p->src = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    if (!p->w || !p->buf || !p->scr || !p->src) return 1;
    for (int j = 0; j < n; ++j) p->w[j] = root_of_unity(j, n, sign);
    return 0;
}

static void plan_free(fft_plan *p)
{
    free(p->w); free(p->buf); free(p->scr); free(p->src);
}

/* one pencil: gather with the given stride, transform, scatter back */
static void pencil(fft_plan *p, cplx *a, long stride, int sign)
{
    for (int j = 0; j < p->n; ++j) p->src[j] = a[j * stride];
    fft_rec(p->n, p->src, 1, p->buf, sign, p->w, 1, p->scr);
    for (int j = 0; j < p->n; ++j) a[j * stride] = p->buf[j];
}

/* sign = -1: a <- (F_{Nz} (x) F_{Ny} (x) F_{Nx}) a  (Def. 2.3 step 2).
 * sign = +1: a <- (F_{Nz}^{-1} (x) F_{Ny}^{-1} (x) F_{Nx}^{-1}) a, including the
 * factor 1/(Nx Ny Nz)  (Def. 2.3 step 4). */
int orc_fft3(int nx, int ny, int nz, double *data, int sign)
{
    if (nx <= 0 || ny <= 0 || nz <= 0 || (sign != 1 && sign != -1)) return 1;
    cplx *a = (cplx *)data;
    fft_plan px, py, pz;
    if (plan_make(&px, nx, sign) || plan_make(&py, ny, sign) || plan_make(&pz, nz, sign)) {
        plan_free(&px); plan_free(&py); plan_free(&pz);
        return 2;
    }
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    for (int l = 0; l < nz; ++l)
        for (int k = 0; k < ny; ++k) pencil(&px, a + l * sz + k * sy, sx, sign);
    for (int l = 0; l < nz; ++l)
        for (int j = 0; j < nx; ++j) pencil(&py, a + l * sz + j, sy, sign);
    for (int k = 0; k < ny; ++k)
        for (int j = 0; j < nx; ++j) pencil(&pz, a + k * sy + j, sz, sign);
    if (sign == 1) {
        const long ns = (long)nx * ny * nz;
        const double inv = 1.0 / (double)ns;
        for (long q = 0; q < ns; ++q) a[q] *= inv;
    }
    plan_free(&px); plan_free(&py); plan_free(&pz);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Wavenumbers, differentiation                                               */
/* ------------------------------------------------------------------------- */

/* Omega_w = nu_w diag(0, 1, ..., n/2 - 1, 0, -n/2 + 1, ..., -1), nu_w = 2 pi/(w_R - w_L)
 * (Sec. 2.3, definition of Lambda_w = i Omega_w; Alg. 2 step 1 with the Nyquist
 * entry 0). */
int orc_wavenumbers(int n, double length, double *omega)
{
    if (n <= 0 || (n % 2) != 0 || !(length > 0)) return 1;
    const double nu = 2.0 * ORC_PI / length;
    for (int m = 0; m < n; ++m) {
        int s;
        if (m < n / 2) s = m;
        else if (m == n / 2) s = 0;
        else s = m - n;
        omega[m] = nu * (double)s;
    }
    return 0;
}

/* (D_w)_{jl} = (1/2) nu_w (-1)^{j+l} cot(nu_w (w_j - w_l)/2) for j != l, 0 on the
 * diagonal (Sec. 2.2).  Row-major n x n. */
int orc_dmatrix(int n, double length, double *D)
{
    if (n <= 0 || (n % 2) != 0 || !(length > 0)) return 1;
    const double nu = 2.0 * ORC_PI / length;
    const double h = length / (double)n;
    for (int j = 0; j < n; ++j)
        for (int l = 0; l < n; ++l) {
            if (j == l) { D[j * n + l] = 0.0; continue; }
            double sgn = ((j + l) % 2 == 0) ? 1.0 : -1.0;
            double arg = nu * ((double)(j - l) * h) / 2.0;
            D[j * n + l] = 0.5 * nu * sgn / tan(arg);
        }
    return 0;
}

/* out = D_axis f on an [nz][ny][nx] real array, computed as F^{-1} (i Omega_axis) F
 * along that axis alone (Sec. 2.3: D = F^{-1} Lambda F, Lambda_w = i Omega_w).
 * axis: 0 = x (D_1), 1 = y (D_2), 2 = z (D_3). */
int orc_deriv(int nx, int ny, int nz, const double *dom, int axis, const double *f, double *out)
{
    if (axis < 0 || axis > 2) return 1;
    const int n = axis == 0 ? nx : (axis == 1 ? ny : nz);
    const double length = dom[2 * axis + 1] - dom[2 * axis];
    double *omega = (double *)malloc(sizeof(double) * (size_t)n);
    fft_plan pf, pb;
    if (!omega || orc_wavenumbers(n, length, omega) || plan_make(&pf, n, -1) || plan_make(&pb, n, 1)) {
        free(omega);
        return 2;
    }
    const long sx = 1, sy = nx, sz = (long)nx * ny;
    const long stride = axis == 0 ? sx : (axis == 1 ? sy : sz);
    cplx *line = (cplx *)malloc(sizeof(cplx) * (size_t)n);
    /* enumerate the pencils: the two other indices */
    int n1 = axis == 0 ? ny : nx, n2 = axis == 2 ? ny : nz;
    long s1 = axis == 0 ? sy : sx, s2 = axis == 2 ? sy : sz;
    for (int b = 0; b < n2; ++b)
        for (int a = 0; a < n1; ++a) {
            long base = a * s1 + b * s2;
            for (int q = 0; q < n; ++q) line[q] = f[base + q * stride];
            pencil(&pf, line, 1, -1);
            for (int q = 0; q < n; ++q) line[q] *= I * omega[q];
            pencil(&pb, line, 1, 1);
            for (int q = 0; q < n; ++q) out[base + q * stride] = creal(line[q]) / (double)n;
        }
    free(line);
    free(omega);
    plan_free(&pf);
    plan_free(&pb);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Propagator coefficients (Prop. 2.2; Alg. 2 steps 2-3)                      */
/* ------------------------------------------------------------------------- */

/* For one wavevector b = (b_x, b_y, b_z) and kappa = t / sqrt(mu eps):
 *   Psi = kappa^2 |b|^2,  r1 = (cos sqrt(Psi) - 1)/Psi,  r2 = sin sqrt(Psi)/sqrt(Psi)
 *   c11 = 1 + kappa^2 (bz^2 + by^2) r1,  c22 = 1 + kappa^2 (bz^2 + bx^2) r1,
 *   c33 = 1 + kappa^2 (by^2 + bx^2) r1,  c12 = -kappa^2 by bx r1,
 *   c13 = -kappa^2 bz bx r1,  c23 = -kappa^2 bz by r1,
 *   s12 = i kappa bz r2,  s13 = i kappa by r2,  s23 = i kappa bx r2.
 * c[6] = {c11, c12, c13, c22, c23, c33}; s[3] = imaginary parts of {s12, s13, s23}. */
void orc_coefficients(double bx, double by, double bz, double kappa, double *c, double *s)
{
    const double Psi = kappa * kappa * (bx * bx + by * by + bz * bz);
    double r1, r2;
    if (Psi == 0.0) {            /* limits of the two quotients */
        r1 = -0.5;
        r2 = 1.0;
    } else {
        const double th = sqrt(Psi);
        r1 = (cos(th) - 1.0) / Psi;
        r2 = sin(th) / th;
    }
    const double k2 = kappa * kappa;
    c[0] = 1.0 + k2 * (bz * bz + by * by) * r1;   /* c11 */
    c[1] = -k2 * by * bx * r1;                    /* c12 */
    c[2] = -k2 * bz * bx * r1;                    /* c13 */
    c[3] = 1.0 + k2 * (bz * bz + bx * bx) * r1;   /* c22 */
    c[4] = -k2 * bz * by * r1;                    /* c23 */
    c[5] = 1.0 + k2 * (by * by + bx * bx) * r1;   /* c33 */
    s[0] = kappa * bz * r2;                       /* s12 / i */
    s[1] = kappa * by * r2;                       /* s13 / i */
    s[2] = kappa * bx * r2;                       /* s23 / i */
}

/* Prop. 2.2 in block form.  On the scaled coefficients (u, v) = (sqrt(mu) H^, sqrt(eps) E^)
 * one mode evolves by the 6x6 matrix
 *       [  C  S ]        C = [c11 c12 c13]        S = [  0    s12  -s13 ]
 *       [ -S  C ]            [c12 c22 c23]            [ -s12   0    s23 ]
 *                            [c13 c23 c33]            [  s13 -s23    0  ]
 * with C real symmetric and S purely imaginary and skew (the s_ij of Prop. 2.2 carry the
 * factor i).  c[6], s[3] are as returned by orc_coefficients. */
static void scaled_block(const double *c, const double *s, cplx M[6][6])
{
    const double C[3][3] = {{c[0], c[1], c[2]}, {c[1], c[3], c[4]}, {c[2], c[4], c[5]}};
    const cplx S[3][3] = {{0, I * s[0], -I * s[1]}, {-I * s[0], 0, I * s[2]}, {I * s[1], -I * s[2], 0}};
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            M[i][j] = C[i][j];
            M[i][3 + j] = S[i][j];
            M[3 + i][j] = -S[i][j];
            M[3 + i][3 + j] = C[i][j];
        }
}

/* y = M x for one mode (6 complex coefficients). */
static void apply_block(cplx M[6][6], const cplx *x, cplx *y)
{
    for (int i = 0; i < 6; ++i) {
        cplx acc = 0;
        for (int j = 0; j < 6; ++j) acc += M[i][j] * x[j];
        y[i] = acc;
    }
}

/* The mode-wise 6x6 map (Hx,Hy,Hz,Ex,Ey,Ez)^ at time 0 -> at time t (Prop. 2.1/2.2,
 * Alg. 2 step 4): the scaled block above, conjugated by the diagonal scaling
 * diag(sqrt(mu) I, sqrt(eps) I).  P is row-major 6x6 complex, interleaved (72 doubles). */
void orc_propagator(double bx, double by, double bz, double t, double mu, double eps, double *P)
{
    double c[6], s[3];
    cplx M[6][6];
    orc_coefficients(bx, by, bz, t / sqrt(mu * eps), c, s);
    scaled_block(c, s, M);
    const double sc[6] = {sqrt(mu), sqrt(mu), sqrt(mu), sqrt(eps), sqrt(eps), sqrt(eps)};
    cplx *out = (cplx *)P;
    for (int i = 0; i < 6; ++i)
        for (int j = 0; j < 6; ++j) out[i * 6 + j] = M[i][j] * sc[j] / sc[i];
}

/* ------------------------------------------------------------------------- */
/* The fully discrete scheme (Def. 2.3, Alg. 1 and Alg. 2)                     */
/* ------------------------------------------------------------------------- */

/* Advance (H, E) by nsteps steps of size tau, each step being Alg. 1 step 4 followed
 * by Alg. 2 with t_end = tau.  H and E are [3][nz][ny][nx] and are overwritten.
 * dom = {xL, xR, yL, yR, zL, zR}.  If max_imag is not NULL it receives the largest
 * |imaginary part| left by the inverse transforms (the exact result is real). */
int orc_step(int nx, int ny, int nz, const double *dom, double mu, double eps, double tau,
             long nsteps, double *H, double *E, double *max_imag)
{
    if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2) return 1;
    if (!(mu > 0) || !(eps > 0) || !isfinite(tau) || nsteps < 0) return 1;
    const long ns = (long)nx * ny * nz;
    const int nn[3] = {nx, ny, nz};
    double *a[3];
    for (int w = 0; w < 3; ++w) {
        a[w] = (double *)malloc(sizeof(double) * (size_t)nn[w]);
        if (!a[w] || orc_wavenumbers(nn[w], dom[2 * w + 1] - dom[2 * w], a[w])) {
            for (int v = 0; v <= w; ++v) free(a[v]);
            return 2;
        }
    }
    /* Alg. 2 steps 2-3: kappa, Psi and the coefficient vectors, computed once */
    const double kappa = tau / sqrt(mu * eps);
    double *cf = (double *)malloc(sizeof(double) * 9 * (size_t)ns);
    cplx *f = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)ns);
    if (!cf || !f) {
        free(cf); free(f);
        for (int w = 0; w < 3; ++w) free(a[w]);
        return 2;
    }
    for (int l = 0; l < nz; ++l)
        for (int k = 0; k < ny; ++k)
            for (int j = 0; j < nx; ++j) {
                long q = ((long)l * ny + k) * nx + j;
                orc_coefficients(a[0][j], a[1][k], a[2][l], kappa, cf + 9 * q, cf + 9 * q + 6);
            }
    const double smu = sqrt(mu), seps = sqrt(eps);
    double mi = 0.0;
    for (long n = 0; n < nsteps; ++n) {
        /* Alg. 1 step 4: transform the six components */
        for (int c = 0; c < 3; ++c)
            for (long q = 0; q < ns; ++q) {
                f[c * ns + q] = H[c * ns + q];
                f[(3 + c) * ns + q] = E[c * ns + q];
            }
        for (int c = 0; c < 6; ++c) orc_fft3(nx, ny, nz, (double *)(f + c * ns), -1);
        /* Alg. 2 step 4: scale to (u, v), apply the mode's block of Prop. 2.2, unscale */
        for (long q = 0; q < ns; ++q) {
            cplx M[6][6], x[6], y[6];
            scaled_block(cf + 9 * q, cf + 9 * q + 6, M);
            for (int c = 0; c < 6; ++c) x[c] = (c < 3 ? smu : seps) * f[c * ns + q];
            apply_block(M, x, y);
            for (int c = 0; c < 6; ++c) f[c * ns + q] = y[c] / (c < 3 ? smu : seps);
        }
        /* Alg. 2 step 5: inverse transform; the result is real up to rounding */
        for (int c = 0; c < 6; ++c) orc_fft3(nx, ny, nz, (double *)(f + c * ns), 1);
        for (int c = 0; c < 3; ++c)
            for (long q = 0; q < ns; ++q) {
                H[c * ns + q] = creal(f[c * ns + q]);
                E[c * ns + q] = creal(f[(3 + c) * ns + q]);
                double im1 = fabs(cimag(f[c * ns + q])), im2 = fabs(cimag(f[(3 + c) * ns + q]));
                if (im1 > mi) mi = im1;
                if (im2 > mi) mi = im2;
            }
    }
    if (max_imag) *max_imag = mi;
    free(cf);
    free(f);
    for (int w = 0; w < 3; ++w) free(a[w]);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Discrete invariants (Sec. 4)                                               */
/* ------------------------------------------------------------------------- */

/* <u, v>_N for real grid functions: the grid mean of u v (Sec. 3 definition).  The sum
 * is compensated (Neumaier) so that it does not add O(n u) of its own to the invariant. */
static double inner(long ns, const double *u, const double *v)
{
    double s = 0.0, comp = 0.0;
    for (long q = 0; q < ns; ++q) {
        const double x = u[q] * v[q];
        const double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x;
        else comp += (x - t) + s;
        s = t;
    }
    return (s + comp) / (double)ns;
}

/* <U, V>_N for 3-component fields [3][ns]: the sum of the three component products. */
static double inner3(long ns, const double *U, const double *V)
{
    return inner(ns, U, V) + inner(ns, U + ns, V + ns) + inner(ns, U + 2 * ns, V + 2 * ns);
}

/* discrete curl of a [3][..] field: (D F)_x = D_2 F_z - D_3 F_y, (D F)_y = D_3 F_x - D_1 F_z,
 * (D F)_z = D_1 F_y - D_2 F_x  (the block matrix D of Sec. 2.2) */
static int curl(int nx, int ny, int nz, const double *dom, const double *F, double *out, double *tmp)
{
    const long ns = (long)nx * ny * nz;
    const int comp[3][2] = {{2, 1}, {0, 2}, {1, 0}};   /* (plus term component, minus term component) */
    const int axp[3] = {1, 2, 0}, axm[3] = {2, 0, 1};     /* derivative axis of plus / minus term */
    for (int c = 0; c < 3; ++c) {
        if (orc_deriv(nx, ny, nz, dom, axp[c], F + comp[c][0] * ns, out + c * ns)) return 1;
        if (orc_deriv(nx, ny, nz, dom, axm[c], F + comp[c][1] * ns, tmp)) return 1;
        for (long q = 0; q < ns; ++q) out[c * ns + q] -= tmp[q];
    }
    return 0;
}

/* Output slots (ORC_NINV doubles):
 *   0 E1          1 E2          2-4 E3[k]     5-7 E4[k]    8-10 E5[k]   11-13 E6[k]
 *  14 H1         15 H2         16-18 M1[w]   19-21 M2[w]
 *  22 ||div~(mu H)||_N   23 ||div~(eps E)||_N   24 max|div~(mu H)|   25 max|div~(eps E)|
 * Definitions: Thm 4.1 (E1..E6, with D_k = D_1, D_2, D_3 for k = 1, 2, 3), Thm 4.3
 * (H1, and the same form on the time derivatives, printed as a second H1, read as
 * H2), Thm 4.4 (M1 = <H, B_k E>_N, M2 = <E, B_k H>_N, B_k = diag(D_k, D_k, D_k)),
 * Thm 4.6 (div~(eps E) = D_1 eps E_x + D_2 eps E_y + D_3 eps E_z; likewise mu H).
 * Time derivatives come from the semi-discrete system (2.4): d/dt H = -(1/mu) D E,
 * d/dt E = (1/eps) D H  (Remark 4.2 gives the same in spectral space). */
#define ORC_NINV 26
int orc_invariants(int nx, int ny, int nz, const double *dom, double mu, double eps,
                   const double *H, const double *E, double *out)
{
    const long ns = (long)nx * ny * nz;
    double *DH = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *DE = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *Hd = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *Ed = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *DHd = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *DEd = (double *)malloc(sizeof(double) * 3 * (size_t)ns);
    double *g = (double *)malloc(sizeof(double) * (size_t)ns);
    double *g2 = (double *)malloc(sizeof(double) * (size_t)ns);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)ns);
    int rc = 0;
    if (!DH || !DE || !Hd || !Ed || !DHd || !DEd || !g || !g2 || !tmp) { rc = 2; goto done; }
    for (int i = 0; i < ORC_NINV; ++i) out[i] = 0.0;

    if (curl(nx, ny, nz, dom, H, DH, tmp) || curl(nx, ny, nz, dom, E, DE, tmp)) { rc = 1; goto done; }
    for (long q = 0; q < 3 * ns; ++q) {
        Hd[q] = -DE[q] / mu;
        Ed[q] = DH[q] / eps;
    }
    if (curl(nx, ny, nz, dom, Hd, DHd, tmp) || curl(nx, ny, nz, dom, Ed, DEd, tmp)) { rc = 1; goto done; }

    /* energies E1, E2 */
    out[0] = 0.5 * mu * inner3(ns, H, H) + 0.5 * eps * inner3(ns, E, E);
    out[1] = 0.5 * mu * inner3(ns, Hd, Hd) + 0.5 * eps * inner3(ns, Ed, Ed);
    /* E3..E6 per derivative direction k */
    for (int k = 0; k < 3; ++k) {
        double e3 = 0, e4 = 0, e5 = 0, e6 = 0;
        for (int c = 0; c < 3; ++c) {
            if (orc_deriv(nx, ny, nz, dom, k, H + c * ns, g)) { rc = 1; goto done; }
            e3 += 0.5 * mu * inner(ns, g, g);
            e5 += 0.5 * mu * inner(ns, H + c * ns, g);
            if (orc_deriv(nx, ny, nz, dom, k, E + c * ns, g)) { rc = 1; goto done; }
            e3 += 0.5 * eps * inner(ns, g, g);
            e5 += 0.5 * eps * inner(ns, E + c * ns, g);
            if (orc_deriv(nx, ny, nz, dom, k, Hd + c * ns, g)) { rc = 1; goto done; }
            e4 += 0.5 * mu * inner(ns, g, g);
            e6 += 0.5 * mu * inner(ns, Hd + c * ns, g);
            if (orc_deriv(nx, ny, nz, dom, k, Ed + c * ns, g)) { rc = 1; goto done; }
            e4 += 0.5 * eps * inner(ns, g, g);
            e6 += 0.5 * eps * inner(ns, Ed + c * ns, g);
        }
        out[2 + k] = e3;
        out[5 + k] = e4;
        out[8 + k] = e5;
        out[11 + k] = e6;
    }
    /* helicities */
    out[14] = inner3(ns, H, DH) / (2.0 * eps) + inner3(ns, E, DE) / (2.0 * mu);
    out[15] = inner3(ns, Hd, DHd) / (2.0 * eps) + inner3(ns, Ed, DEd) / (2.0 * mu);
    /* momenta, one value per derivative direction */
    for (int k = 0; k < 3; ++k) {
        double m1 = 0, m2 = 0;
        for (int c = 0; c < 3; ++c) {
            if (orc_deriv(nx, ny, nz, dom, k, E + c * ns, g)) { rc = 1; goto done; }
            m1 += inner(ns, H + c * ns, g);
            if (orc_deriv(nx, ny, nz, dom, k, H + c * ns, g)) { rc = 1; goto done; }
            m2 += inner(ns, E + c * ns, g);
        }
        out[16 + k] = m1;
        out[19 + k] = m2;
    }
    /* divergences of mu H and eps E */
    for (int which = 0; which < 2; ++which) {
        const double *F = which == 0 ? H : E;
        const double coef = which == 0 ? mu : eps;
        for (long q = 0; q < ns; ++q) g2[q] = 0.0;
        for (int c = 0; c < 3; ++c) {
            for (long q = 0; q < ns; ++q) tmp[q] = coef * F[c * ns + q];
            if (orc_deriv(nx, ny, nz, dom, c, tmp, g)) { rc = 1; goto done; }
            for (long q = 0; q < ns; ++q) g2[q] += g[q];
        }
        double mx = 0.0;
        for (long q = 0; q < ns; ++q)
            if (fabs(g2[q]) > mx) mx = fabs(g2[q]);
        out[22 + which] = sqrt(inner(ns, g2, g2));
        out[24 + which] = mx;
    }
done:
    free(DH); free(DE); free(Hd); free(Ed); free(DHd); free(DEd); free(g); free(g2); free(tmp);
    return rc;
}

/* omega(U, V) = <E_U, H_V>_N - <E_V, H_U>_N summed over components: the bilinear form
 * whose conservation is the discrete statement of Thm 4.5 (dE ^ dH preserved). */
double orc_symplectic(int nx, int ny, int nz, const double *HU, const double *EU,
                      const double *HV, const double *EV)
{
    const long n3 = 3L * nx * ny * nz;
    double a = 0.0, b = 0.0;
    for (long q = 0; q < n3; ++q) {
        a += EU[q] * HV[q];
        b += EV[q] * HU[q];
    }
    return (a - b) / ((double)nx * ny * nz);
}

int orc_num_invariants(void) { return ORC_NINV; }

/* Drift scales of a state: the Cauchy-Schwarz bounds of the invariants that can be near
 * zero (H1, M1_k, the divergence norms), as plain sums over the full 3-D DFT of the six
 * components.  Parseval with the grid mean of Sec. 3: every term is divided by N_S^2.
 *   out[0]    sum |b| (|H^|^2/(2 eps) + |E^|^2/(2 mu))          bounds |H1|   (Thm 4.3)
 *   out[1..3] sqrt(sum |H^|^2) sqrt(sum b_k^2 |E^|^2)           bounds |M1_k| (Thm 4.4)
 *   out[4]    mu sqrt(sum |b|^2 |H^|^2), out[5] the same for eps, E
 *                                                   bound the divergence norms (Thm 4.6)
 * with b = (Omega_x, Omega_y, Omega_z) of Sec. 2.3 (Nyquist entries 0). */
int orc_drift_scales(int nx, int ny, int nz, const double *dom, double mu, double eps,
                     const double *H, const double *E, double *out)
{
    if (nx < 2 || ny < 2 || nz < 2 || nx % 2 || ny % 2 || nz % 2 || !(mu > 0) || !(eps > 0)) return 1;
    const long ns = (long)nx * ny * nz;
    const int nn[3] = {nx, ny, nz};
    double *a[3] = {NULL, NULL, NULL};
    cplx *f = (cplx *)malloc(sizeof(cplx) * 6 * (size_t)ns);
    int rc = f ? 0 : 2;
    for (int w = 0; w < 3 && !rc; ++w) {
        a[w] = (double *)malloc(sizeof(double) * (size_t)nn[w]);
        if (!a[w] || orc_wavenumbers(nn[w], dom[2 * w + 1] - dom[2 * w], a[w])) rc = 2;
    }
    if (!rc) {
        for (int c = 0; c < 3; ++c)
            for (long q = 0; q < ns; ++q) {
                f[c * ns + q] = H[c * ns + q];
                f[(3 + c) * ns + q] = E[c * ns + q];
            }
        for (int c = 0; c < 6; ++c) orc_fft3(nx, ny, nz, (double *)(f + c * ns), -1);
        double sh = 0.0, hh = 0.0, be[3] = {0.0, 0.0, 0.0}, b2h = 0.0, b2e = 0.0;
        const double n2 = (double)ns * (double)ns;
        for (int l = 0; l < nz; ++l)
            for (int k = 0; k < ny; ++k)
                for (int j = 0; j < nx; ++j) {
                    const long q = ((long)l * ny + k) * nx + j;
                    const double b[3] = {a[0][j], a[1][k], a[2][l]};
                    const double bb = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
                    double h2 = 0.0, e2 = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        h2 += creal(f[c * ns + q] * conj(f[c * ns + q]));
                        e2 += creal(f[(3 + c) * ns + q] * conj(f[(3 + c) * ns + q]));
                    }
                    h2 /= n2;
                    e2 /= n2;
                    sh += sqrt(bb) * (h2 / (2.0 * eps) + e2 / (2.0 * mu));
                    hh += h2;
                    for (int w = 0; w < 3; ++w) be[w] += b[w] * b[w] * e2;
                    b2h += bb * h2;
                    b2e += bb * e2;
                }
        out[0] = sh;
        for (int w = 0; w < 3; ++w) out[1 + w] = sqrt(hh) * sqrt(be[w]);
        out[4] = mu * sqrt(b2h);
        out[5] = eps * sqrt(b2e);
    }
    free(f);
    for (int w = 0; w < 3; ++w) free(a[w]);
    return rc;
}
