/*
 * FP64 CPU oracle for semi-Lagrangian Gauss-Newton-Krylov diffeomorphic
 * registration (Mang, Gholami, Biros, "Distributed-memory large deformation
 * diffeomorphic 3D image registration", SC16).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library. The GPU library never
 * links, includes or calls anything here, and this file includes nothing
 * from it.
 *
 * Everything is plain double-precision loops (OpenMP over grid points or
 * lines), with this file's own FFT (recursive mixed radix) and its own
 * tricubic Lagrange interpolation (a 64-term triple sum). Where the GPU path
 * uses an algebraically equivalent but cleverer form (line FFTs, fused
 * interpolation of a combined field, separable stencils) this oracle keeps
 * the plain form, so that agreement tests the equivalence.
 *
 * Conventions (paper section III-B1, "Space"):
 *   domain [0, 2*pi)^3, periodic; grid x_i = 2*pi*i/N, i = 0..N-1;
 *   arrays are C-order [N1][N2][N3] (x3 fastest); vector fields are
 *   three such arrays back to back.
 *   Forward DFT uses exp(-i k.x); wavenumber k_j = m for m <= N/2 else m-N.
 *   Odd symbols (derivatives, the k in the Leray projection) use k~ with
 *   the Nyquist wavenumber N/2 set to zero; even symbols use the full k.
 *   Semi-Lagrangian points are stored as displacements D in cell units:
 *   X = x + h*D per axis.
 *   Inner product <u,w> = h1*h2*h3 * sum u*w (the L2 inner product on the grid).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

#define TWO_PI 6.283185307179586476925286766559

/* ------------------------------------------------------------------ */
/* grid helpers                                                        */
/* ------------------------------------------------------------------ */

static long npts(const int *n) { return (long)n[0] * n[1] * n[2]; }

static long pmod(long a, long m) {
    long r = a % m;
    return r < 0 ? r + m : r;
}

static long at(const int *n, long i1, long i2, long i3) {
    return (i1 * n[1] + i2) * n[2] + i3;
}

/* wavenumber of DFT index m on an axis of length nn (section III-B1) */
static double wavenum(int m, int nn) { return (2 * m <= nn) ? (double)m : (double)(m - nn); }

/* the same with the Nyquist wavenumber removed, for odd (derivative) symbols */
static double wavenum_odd(int m, int nn) { return (2 * m == nn) ? 0.0 : wavenum(m, nn); }

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}

static double dot_raw(long len, const double *a, const double *b) {
    double s = 0.0;
    for (long i = 0; i < len; i++) s += a[i] * b[i];
    return s;
}

/* <u,w> = h1 h2 h3 sum_i u_i w_i over ncomp components */
static double inner(const int *n, int ncomp, const double *u, const double *w) {
    double h3 = (TWO_PI / n[0]) * (TWO_PI / n[1]) * (TWO_PI / n[2]);
    return h3 * dot_raw(ncomp * npts(n), u, w);
}

/* ------------------------------------------------------------------ */
/* FFT: recursive decimation in time over the smallest prime factor     */
/* ------------------------------------------------------------------ */

static int smallest_factor(int n) {
    for (int p = 2; p * p <= n; p++)
        if (n % p == 0) return p;
    return n;
}

/* y[k] = sum_j x[j*s] * w_n^(j*k), k = 0..n-1, with w_n = exp(sign*2*pi*i/n).
 * tw[j] = exp(sign*2*pi*i*j/ntop) and n divides ntop. work holds 2*n values. */
static void dft_rec(const cplx *x, long s, cplx *y, int n, const cplx *tw, int ntop, cplx *work) {
    if (n == 1) {
        y[0] = x[0];
        return;
    }
    int p = smallest_factor(n), m = n / p;
    long step = ntop / n;
    if (m == 1) { /* prime length: the defining sum */
        for (int k = 0; k < n; k++) {
            cplx acc = 0;
            for (int j = 0; j < n; j++) acc += x[j * s] * tw[((long)j * k % n) * step];
            y[k] = acc;
        }
        return;
    }
    /* sub[r*m + q] = length-m DFT of x[(p*q + r)*s], q = 0..m-1 */
    cplx *sub = work;
    for (int r = 0; r < p; r++) dft_rec(x + r * s, s * p, sub + (long)r * m, m, tw, ntop, work + n);
    /* X[k] = sum_r w_n^(r*k) * sub_r[k mod m] */
    for (int k = 0; k < n; k++) {
        cplx acc = 0;
        for (int r = 0; r < p; r++) acc += tw[((long)r * k % n) * step] * sub[(long)r * m + k % m];
        y[k] = acc;
    }
}

/* unnormalised DFT of every line along one axis, in place */
static void fft_axis(cplx *a, const int *n, int axis, int sign) {
    int len = n[axis];
    long stride = axis == 2 ? 1 : (axis == 1 ? n[2] : (long)n[1] * n[2]);
    long nlines = npts(n) / len;
    cplx *tw = xmalloc(sizeof(cplx) * len);
    for (int j = 0; j < len; j++) {
        double ang = TWO_PI * j / len;
        tw[j] = cos(ang) + I * (sign * sin(ang));
    }
#pragma omp parallel
    {
        cplx *in = xmalloc(sizeof(cplx) * len), *out = xmalloc(sizeof(cplx) * len);
        cplx *work = xmalloc(sizeof(cplx) * 2 * len);
#pragma omp for schedule(static)
        for (long l = 0; l < nlines; l++) {
            long base;
            if (axis == 2) base = l * n[2];
            else if (axis == 1) base = (l / n[2]) * (long)n[1] * n[2] + l % n[2];
            else base = l;
            for (int j = 0; j < len; j++) in[j] = a[base + j * stride];
            dft_rec(in, 1, out, len, tw, len, work);
            for (int j = 0; j < len; j++) a[base + j * stride] = out[j];
        }
        free(in);
        free(out);
        free(work);
    }
    free(tw);
}

/* 3D DFT (sign -1 forward, unnormalised; sign +1 inverse, divided by N1 N2 N3) */
static void fft3(cplx *a, const int *n, int sign) {
    fft_axis(a, n, 2, sign);
    fft_axis(a, n, 1, sign);
    fft_axis(a, n, 0, sign);
    if (sign > 0) {
        double s = 1.0 / npts(n);
        long N = npts(n);
        for (long i = 0; i < N; i++) a[i] *= s;
    }
}

static cplx *spec_of(const int *n, const double *u) {
    long N = npts(n);
    cplx *a = xmalloc(sizeof(cplx) * N);
    for (long i = 0; i < N; i++) a[i] = u[i];
    fft3(a, n, -1);
    return a;
}

/* inverse transform and keep the real part; frees the spectrum */
static void real_of(const int *n, cplx *a, double *u) {
    long N = npts(n);
    fft3(a, n, +1);
    for (long i = 0; i < N; i++) u[i] = creal(a[i]);
    free(a);
}

/* exported complex 3D DFT on interleaved (re, im) doubles, for the FFT pins */
void oracle_fft3(const int *n, const double *in, double *out, int sign) {
    long N = npts(n);
    cplx *a = xmalloc(sizeof(cplx) * N);
    for (long i = 0; i < N; i++) a[i] = in[2 * i] + I * in[2 * i + 1];
    fft3(a, n, sign);
    for (long i = 0; i < N; i++) {
        out[2 * i] = creal(a[i]);
        out[2 * i + 1] = cimag(a[i]);
    }
    free(a);
}

/* ------------------------------------------------------------------ */
/* spectral operators (section III-B1; Leray operator of eq. (4);      */
/* preconditioner of section III-A)                                     */
/* ------------------------------------------------------------------ */

/* wavenumbers of flat spectral index p */
static void kvec(const int *n, long p, double k[3], double kt[3]) {
    int m3 = (int)(p % n[2]);
    int m2 = (int)((p / n[2]) % n[1]);
    int m1 = (int)(p / ((long)n[1] * n[2]));
    k[0] = wavenum(m1, n[0]);
    k[1] = wavenum(m2, n[1]);
    k[2] = wavenum(m3, n[2]);
    kt[0] = wavenum_odd(m1, n[0]);
    kt[1] = wavenum_odd(m2, n[1]);
    kt[2] = wavenum_odd(m3, n[2]);
}

/* partial derivative along axis j: symbol i*k~_j */
void oracle_deriv(const int *n, int j, const double *u, double *du) {
    long N = npts(n);
    cplx *a = spec_of(n, u);
    for (long p = 0; p < N; p++) {
        double k[3], kt[3];
        kvec(n, p, k, kt);
        a[p] *= I * kt[j];
    }
    real_of(n, a, du);
}

/* gradient of a scalar: g[j] = d_j u */
void oracle_grad(const int *n, const double *u, double *g) {
    long N = npts(n);
    for (int j = 0; j < 3; j++) oracle_deriv(n, j, u, g + j * N);
}

/* divergence of a vector field: sum_j i k~_j v^_j */
void oracle_div(const int *n, const double *v, double *dv) {
    long N = npts(n);
    cplx *acc = xmalloc(sizeof(cplx) * N);
    for (long p = 0; p < N; p++) acc[p] = 0;
    for (int j = 0; j < 3; j++) {
        cplx *a = spec_of(n, v + j * N);
        for (long p = 0; p < N; p++) {
            double k[3], kt[3];
            kvec(n, p, k, kt);
            acc[p] += I * kt[j] * a[p];
        }
        free(a);
    }
    real_of(n, acc, dv);
}

/* apply P^ = I - k~ k~^T / |k~|^2 (I where k~ = 0) to a spectral vector */
static void leray_hat(const int *n, cplx *a0, cplx *a1, cplx *a2) {
    long N = npts(n);
    for (long p = 0; p < N; p++) {
        double k[3], kt[3];
        kvec(n, p, k, kt);
        double kk = kt[0] * kt[0] + kt[1] * kt[1] + kt[2] * kt[2];
        if (kk == 0.0) continue;
        cplx kd = (kt[0] * a0[p] + kt[1] * a1[p] + kt[2] * a2[p]) / kk;
        a0[p] -= kt[0] * kd;
        a1[p] -= kt[1] * kd;
        a2[p] -= kt[2] * kd;
    }
}

/* Leray projection P = I - grad lap^-1 div (eq. (4)) */
void oracle_leray(const int *n, const double *v, double *pv) {
    long N = npts(n);
    cplx *a[3];
    for (int j = 0; j < 3; j++) a[j] = spec_of(n, v + j * N);
    leray_hat(n, a[0], a[1], a[2]);
    for (int j = 0; j < 3; j++) real_of(n, a[j], pv + j * N);
}

/* componentwise multiplication by a real even symbol */
enum { SYM_BIHARM = 0, SYM_INVBIHARM = 1, SYM_GAUSS = 2, SYM_LAPLACE = 3 };

static double even_symbol(int which, const double k[3], double par) {
    double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    switch (which) {
    case SYM_BIHARM: return par * k2 * k2;                     /* par*Lap^2: beta |k|^4 */
    case SYM_INVBIHARM: return k2 == 0.0 ? 1.0 : 1.0 / (par * k2 * k2);
    case SYM_GAUSS: return exp(-0.5 * par * par * k2);          /* par = sigma (radians) */
    case SYM_LAPLACE: return -k2;
    }
    return 0.0;
}

void oracle_even_op(const int *n, int ncomp, int which, double par, const double *u, double *out) {
    long N = npts(n);
    for (int c = 0; c < ncomp; c++) {
        cplx *a = spec_of(n, u + c * N);
        for (long p = 0; p < N; p++) {
            double k[3], kt[3];
            kvec(n, p, k, kt);
            a[p] *= even_symbol(which, k, par);
        }
        real_of(n, a, out + c * N);
    }
}

/* spectral preconditioner (section III-A): z^ = r^/(beta |k|^4), z^_0 = r^_0,
 * then the Leray projection in the isochoric case */
void oracle_precond(const int *n, double beta, int isochoric, const double *r, double *z) {
    long N = npts(n);
    cplx *a[3];
    for (int j = 0; j < 3; j++) {
        a[j] = spec_of(n, r + j * N);
        for (long p = 0; p < N; p++) {
            double k[3], kt[3];
            kvec(n, p, k, kt);
            a[j][p] *= even_symbol(SYM_INVBIHARM, k, beta);
        }
    }
    if (isochoric) leray_hat(n, a[0], a[1], a[2]);
    for (int j = 0; j < 3; j++) real_of(n, a[j], z + j * N);
}

/* out = IFFT(beta |k|^4 x^ + P^ y^)  (the assembly in eqs. (4) and (5e)) */
static void assemble(const int *n, double beta, int isochoric, const double *x, const double *y,
                     double *out) {
    long N = npts(n);
    cplx *a[3];
    for (int j = 0; j < 3; j++) a[j] = spec_of(n, y + j * N);
    if (isochoric) leray_hat(n, a[0], a[1], a[2]);
    for (int j = 0; j < 3; j++) {
        cplx *b = spec_of(n, x + j * N);
        for (long p = 0; p < N; p++) {
            double k[3], kt[3];
            kvec(n, p, k, kt);
            a[j][p] += even_symbol(SYM_BIHARM, k, beta) * b[p];
        }
        free(b);
        real_of(n, a[j], out + j * N);
    }
}

/* regulariser 1/2 beta ||lap v||^2 by Parseval: (2pi)^3/(N)^2 sum |k|^4 |v^|^2 */
static double regulariser(const int *n, double beta, const double *v) {
    long N = npts(n);
    double s = 0.0;
    for (int j = 0; j < 3; j++) {
        cplx *a = spec_of(n, v + j * N);
        for (long p = 0; p < N; p++) {
            double k[3], kt[3];
            kvec(n, p, k, kt);
            double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
            s += k2 * k2 * (creal(a[p]) * creal(a[p]) + cimag(a[p]) * cimag(a[p]));
        }
        free(a);
    }
    double vol = TWO_PI * TWO_PI * TWO_PI;
    return 0.5 * beta * vol * s / ((double)N * (double)N);
}

double oracle_regulariser(const int *n, double beta, const double *v) { return regulariser(n, beta, v); }

/* spectral resampling between grids n (source) and m (target), per component.
 * Keeps modes with |k_j| < min(n_j, m_j)/2 and drops the Nyquist planes. The
 * unnormalised DFT coefficients are scaled by M/N so that the represented
 * trigonometric polynomial is unchanged. */
void oracle_resample(const int *n, const int *m, int ncomp, const double *u, double *out) {
    long N = npts(n), M = npts(m);
    for (int c = 0; c < ncomp; c++) {
        cplx *a = spec_of(n, u + c * N);
        cplx *b = xmalloc(sizeof(cplx) * M);
        for (long q = 0; q < M; q++) b[q] = 0;
        for (long p = 0; p < N; p++) {
            int i3 = (int)(p % n[2]), i2 = (int)((p / n[2]) % n[1]), i1 = (int)(p / ((long)n[1] * n[2]));
            int kk[3] = {(int)wavenum(i1, n[0]), (int)wavenum(i2, n[1]), (int)wavenum(i3, n[2])};
            int keep = 1;
            long t[3];
            for (int j = 0; j < 3; j++) {
                int lim = n[j] < m[j] ? n[j] : m[j];
                if (2 * abs(kk[j]) >= lim) keep = 0;
                t[j] = kk[j] < 0 ? kk[j] + m[j] : kk[j];
            }
            if (keep) b[at(m, t[0], t[1], t[2])] = a[p] * ((double)M / (double)N);
        }
        free(a);
        real_of(m, b, out + c * M);
    }
}

/* ------------------------------------------------------------------ */
/* tricubic Lagrange interpolation (section III-B2 and III-C2)          */
/* ------------------------------------------------------------------ */

/* cubic Lagrange basis on the nodes -1, 0, 1, 2 evaluated at t */
static void lagrange4(double t, double w[4]) {
    w[0] = -t * (t - 1.0) * (t - 2.0) / 6.0;
    w[1] = (t + 1.0) * (t - 1.0) * (t - 2.0) / 2.0;
    w[2] = -(t + 1.0) * t * (t - 2.0) / 2.0;
    w[3] = (t + 1.0) * t * (t - 1.0) / 6.0;
}

/* out(x_i) = f(x_i + h*D_i): the 64-term sum over the periodic stencil
 * m-1..m+2 per axis, with m = floor(i + D) and t = i + D - m. */
void oracle_interp(const int *n, const double *f, const double *D, double *out) {
    long N = npts(n);
#pragma omp parallel for schedule(static)
    for (long p = 0; p < N; p++) {
        long ii[3] = {p / ((long)n[1] * n[2]), (p / n[2]) % n[1], p % n[2]};
        long m[3];
        double w[3][4];
        for (int j = 0; j < 3; j++) {
            double s = (double)ii[j] + D[j * N + p];
            double fl = floor(s);
            m[j] = (long)fl;
            lagrange4(s - fl, w[j]);
        }
        double acc = 0.0;
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++)
                for (int c = 0; c < 4; c++)
                    acc += w[0][a] * w[1][b] * w[2][c] *
                           f[at(n, pmod(m[0] + a - 1, n[0]), pmod(m[1] + b - 1, n[1]), pmod(m[2] + c - 1, n[2]))];
        out[p] = acc;
    }
}

/* transpose of the interpolation operator: out += sum over targets of the
 * same 64 weights times g (a scatter-add; serial, for small grids) */
void oracle_interp_transpose(const int *n, const double *g, const double *D, double *out) {
    long N = npts(n);
    for (long p = 0; p < N; p++) out[p] = 0.0;
    for (long p = 0; p < N; p++) {
        long ii[3] = {p / ((long)n[1] * n[2]), (p / n[2]) % n[1], p % n[2]};
        long m[3];
        double w[3][4];
        for (int j = 0; j < 3; j++) {
            double s = (double)ii[j] + D[j * N + p];
            double fl = floor(s);
            m[j] = (long)fl;
            lagrange4(s - fl, w[j]);
        }
        for (int a = 0; a < 4; a++)
            for (int b = 0; b < 4; b++)
                for (int c = 0; c < 4; c++)
                    out[at(n, pmod(m[0] + a - 1, n[0]), pmod(m[1] + b - 1, n[1]), pmod(m[2] + c - 1, n[2]))] +=
                        w[0][a] * w[1][b] * w[2][c] * g[p];
    }
}

/* ------------------------------------------------------------------ */
/* RK2 characteristics (eq. (6))                                        */
/* ------------------------------------------------------------------ */

/* Departure points of the velocity sign*v over one step dt = 1/nt:
 *   X* = x - dt u(x),  X = x - dt/2 (u(x) + u(X*)),  u = sign*v,
 * returned as D = (X - x)/h per axis. */
void oracle_backtrace(const int *n, int nt, const double *v, double sign, double *D) {
    long N = npts(n);
    double dt = 1.0 / nt;
    double *Ds = xmalloc(sizeof(double) * 3 * N), *w = xmalloc(sizeof(double) * 3 * N);
    for (int j = 0; j < 3; j++) {
        double h = TWO_PI / n[j];
        for (long p = 0; p < N; p++) Ds[j * N + p] = -dt * sign * v[j * N + p] / h;
    }
    for (int j = 0; j < 3; j++) oracle_interp(n, v + j * N, Ds, w + j * N);
    for (int j = 0; j < 3; j++) {
        double h = TWO_PI / n[j];
        for (long p = 0; p < N; p++) D[j * N + p] = -dt * sign * (v[j * N + p] + w[j * N + p]) / (2.0 * h);
    }
    free(Ds);
    free(w);
}

/* ------------------------------------------------------------------ */
/* transport solves (eqs. (2b), (3), (5a), (5c) with the RK2 scheme     */
/* of eq. (7))                                                          */
/* ------------------------------------------------------------------ */

/* state: rho^{n+1}(x) = rho^n(X); hist holds rho^0..rho^nt */
void oracle_state(const int *n, int nt, const double *Df, const double *rho0, double *hist) {
    long N = npts(n);
    memcpy(hist, rho0, sizeof(double) * N);
    for (int k = 0; k < nt; k++) oracle_interp(n, hist + k * N, Df, hist + (k + 1) * N);
}

/* One backward step (in tau = 1 - t) of -d_t nu - div(v nu) = 0, written
 * as d_tau nu + (-v).grad nu = nu * div v and advanced with eq. (7):
 *   nu0 = nu(X), f0 = nu0 c(X), nu* = nu0 + dt f0, f* = nu* c(x),
 *   nu_new = nu0 + dt/2 (f0 + f*).
 * c = div v on the grid, cX = c interpolated at X (once per plan); both
 * NULL when div v = 0 is enforced, and then the step is a pure interpolation. */
static void adjoint_step(const int *n, double dt, const double *Da, const double *c, const double *cX,
                         const double *nu, double *out) {
    long N = npts(n);
    oracle_interp(n, nu, Da, out);
    if (!c) return;
    for (long p = 0; p < N; p++) {
        double nu0 = out[p];
        double f0 = nu0 * cX[p];
        double nus = nu0 + dt * f0;
        double fs = nus * c[p];
        out[p] = nu0 + 0.5 * dt * (f0 + fs);
    }
}

/* trapezoid weights on t^0..t^nt */
static double trap_w(int k, int nt) { return (k == 0 || k == nt) ? 0.5 / nt : 1.0 / nt; }

/* adjoint history lam^nt..lam^0 from lam^nt = lam1 (hist holds nt+1 slices,
 * index = time level) */
void oracle_adjoint(const int *n, int nt, const double *Da, const double *c, const double *cX,
                    const double *lam1, double *hist) {
    long N = npts(n);
    double dt = 1.0 / nt;
    memcpy(hist + (long)nt * N, lam1, sizeof(double) * N);
    for (int k = nt; k > 0; k--) adjoint_step(n, dt, Da, c, cX, hist + (long)k * N, hist + (long)(k - 1) * N);
}

/* ------------------------------------------------------------------ */
/* reduced gradient, Gauss-Newton Hessian, deformation                   */
/* ------------------------------------------------------------------ */

typedef struct {
    int32_t n[3];
    int32_t nt;
    double beta, beta_final, beta_factor;
    int32_t isochoric;
    int32_t forcing; /* 0: eta = min(0.5, r), 1: eta = min(0.5, sqrt(r)), r = |g|/|g0| */
    double gtol, mismatch_tol;
    int32_t max_newton, max_pcg, max_ls;
    int32_t hessian; /* 0: Gauss-Newton (the paper's runs), 1: full Newton */
    double armijo_c1;
    /* Continuation and stopping (section III-A leaves both to the
     * application): gtol_level > 0 solves the levels above beta_final only
     * to |g| <= gtol_level * ref; gnorm_ref > 0 makes ref (and the forcing
     * ratio) absolute instead of |g0| of the level. */
    double gtol_level, gnorm_ref;
    /* > 0: the gradient reference of the first continuation level, in place
     * of its first gradient norm (grid continuation: the level started on a
     * coarser grid, whose first gradient norm this is) */
    double gref_first;
} oracle_params;

/* everything the gradient and the Hessian need at one velocity */
typedef struct {
    int n[3], nt, iso;
    long N;
    double *Df, *Da;   /* plans for v and -v: 3N each */
    double *rho;       /* rho^0..rho^nt */
    double *grho;      /* grad rho^n: (nt+1) * 3N */
    double *c, *cX;    /* div v and its value at X_a (NULL if isochoric) */
} oracle_state_t;

static void st_free(oracle_state_t *s) {
    free(s->Df);
    free(s->Da);
    free(s->rho);
    free(s->grho);
    free(s->c);
    free(s->cX);
    memset(s, 0, sizeof(*s));
}

/* plan + state solve (enough for the objective) */
static void st_forward(oracle_state_t *s, const int *n, int nt, int iso, const double *v, const double *rhoT) {
    memset(s, 0, sizeof(*s));
    memcpy(s->n, n, sizeof(int) * 3);
    s->nt = nt;
    s->iso = iso;
    s->N = npts(n);
    s->Df = xmalloc(sizeof(double) * 3 * s->N);
    oracle_backtrace(n, nt, v, +1.0, s->Df);
    s->rho = xmalloc(sizeof(double) * (nt + 1) * s->N);
    oracle_state(n, nt, s->Df, rhoT, s->rho);
}

/* the rest of what the adjoint and incremental solves need */
static void st_complete(oracle_state_t *s, const double *v) {
    long N = s->N;
    int nt = s->nt;
    s->Da = xmalloc(sizeof(double) * 3 * N);
    oracle_backtrace(s->n, nt, v, -1.0, s->Da);
    s->grho = xmalloc(sizeof(double) * (nt + 1) * 3 * N);
    for (int k = 0; k <= nt; k++) oracle_grad(s->n, s->rho + (long)k * N, s->grho + (long)k * 3 * N);
    if (!s->iso) {
        s->c = xmalloc(sizeof(double) * N);
        s->cX = xmalloc(sizeof(double) * N);
        oracle_div(s->n, v, s->c);
        oracle_interp(s->n, s->c, s->Da, s->cX);
    }
}

static double objective(const oracle_state_t *s, double beta, const double *v, const double *rhoT,
                        const double *rhoR, double *mismatch) {
    long N = s->N;
    const double *r1 = s->rho + (long)s->nt * N;
    double *d = xmalloc(sizeof(double) * N), *d0 = xmalloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) {
        d[p] = r1[p] - rhoR[p];
        d0[p] = rhoT[p] - rhoR[p];
    }
    double dd = inner(s->n, 1, d, d), d00 = inner(s->n, 1, d0, d0);
    if (mismatch) *mismatch = d00 > 0 ? sqrt(dd / d00) : 0.0;
    free(d);
    free(d0);
    return 0.5 * dd + regulariser(s->n, beta, v);
}

/* b = sum_n w_n lam^n grad rho^n over an adjoint history */
static void accumulate_b(const oracle_state_t *s, const double *lam, double *b) {
    long N = s->N;
    int nt = s->nt;
    memset(b, 0, sizeof(double) * 3 * N);
    for (int k = 0; k <= nt; k++) {
        double w = trap_w(k, nt);
        for (int j = 0; j < 3; j++)
            for (long p = 0; p < N; p++) b[j * N + p] += w * lam[(long)k * N + p] * s->grho[(long)k * 3 * N + j * N + p];
    }
}

/* g = beta lap^2 v + P b with b = int lam grad rho dt (eq. (4)); the
 * adjoint history is copied to lam_out when it is not NULL */
static void gradient_from_state(const oracle_state_t *s, double beta, const double *v, const double *rhoR,
                                double *g, double *lam_out) {
    long N = s->N;
    int nt = s->nt;
    double *lam = xmalloc(sizeof(double) * (nt + 1) * N);
    double *lam1 = xmalloc(sizeof(double) * N);
    const double *r1 = s->rho + (long)nt * N;
    for (long p = 0; p < N; p++) lam1[p] = rhoR[p] - r1[p];
    oracle_adjoint(s->n, nt, s->Da, s->c, s->cX, lam1, lam);
    if (lam_out) memcpy(lam_out, lam, sizeof(double) * (nt + 1) * N);
    double *b = xmalloc(sizeof(double) * 3 * N);
    accumulate_b(s, lam, b);
    assemble(s->n, beta, s->iso, v, b, g);
    free(lam);
    free(lam1);
    free(b);
}

/* Gauss-Newton Hessian matvec (eqs. (5a)-(5e) without the lambda terms) */
static void hessian_from_state(const oracle_state_t *s, double beta, const double *vt, double *Hvt) {
    long N = s->N;
    int nt = s->nt;
    double dt = 1.0 / nt;
    /* s^n = vt . grad rho^n, for the source f = -s of the incremental state */
    double *src = xmalloc(sizeof(double) * (nt + 1) * N);
    for (int k = 0; k <= nt; k++)
        for (long p = 0; p < N; p++) {
            const double *gr = s->grho + (long)k * 3 * N;
            src[(long)k * N + p] = -(vt[p] * gr[p] + vt[N + p] * gr[N + p] + vt[2 * N + p] * gr[2 * N + p]);
        }
    /* incremental state with eq. (7); f does not depend on the unknown, so
     * the predictor is not needed: nu0 = rt(X), f0 = f^n(X), f* = f^{n+1}(x) */
    double *rt = xmalloc(sizeof(double) * N), *nu0 = xmalloc(sizeof(double) * N), *f0 = xmalloc(sizeof(double) * N);
    memset(rt, 0, sizeof(double) * N);
    for (int k = 0; k < nt; k++) {
        oracle_interp(s->n, rt, s->Df, nu0);
        oracle_interp(s->n, src + (long)k * N, s->Df, f0);
        for (long p = 0; p < N; p++) rt[p] = nu0[p] + 0.5 * dt * (f0[p] + src[(long)(k + 1) * N + p]);
    }
    /* incremental adjoint from lam~(1) = -rho~(1), same operator as the adjoint */
    double *lam = xmalloc(sizeof(double) * (nt + 1) * N);
    for (long p = 0; p < N; p++) rt[p] = -rt[p];
    oracle_adjoint(s->n, nt, s->Da, s->c, s->cX, rt, lam);
    double *bt = xmalloc(sizeof(double) * 3 * N);
    accumulate_b(s, lam, bt);
    assemble(s->n, beta, s->iso, vt, bt, Hvt);
    free(src);
    free(rt);
    free(nu0);
    free(f0);
    free(lam);
    free(bt);
}

/* Full Newton Hessian matvec (eqs. (5a)-(5e) with every term): the
 * incremental adjoint carries the source div(lam vt) of eq. (5c), and b~
 * gains the term int lam grad rho~ dt. lam is the adjoint history of the
 * gradient at the same v (levels 0..nt). Each step of the incremental
 * adjoint is eq. (7) written out with f(nu, x, tau) = nu c(x) + s(x, tau),
 * s = div(lam vt) at the step's two time levels:
 *   nu0 = nu(X), f0 = nu0 c(X) + s^k(X), nu* = nu0 + dt f0,
 *   f* = nu* c(x) + s^{k-1}(x), nu_new = nu0 + dt/2 (f0 + f*). */
static void newton_from_state(const oracle_state_t *s, double beta, const double *lamg, const double *vt,
                              double *Hvt) {
    long N = s->N;
    int nt = s->nt;
    double dt = 1.0 / nt;
    /* incremental state history rho~^0..rho~^nt with f = -vt . grad rho */
    double *src = xmalloc(sizeof(double) * (nt + 1) * N);
    for (int k = 0; k <= nt; k++)
        for (long p = 0; p < N; p++) {
            const double *gr = s->grho + (long)k * 3 * N;
            src[(long)k * N + p] = -(vt[p] * gr[p] + vt[N + p] * gr[N + p] + vt[2 * N + p] * gr[2 * N + p]);
        }
    double *rt = xmalloc(sizeof(double) * (nt + 1) * N), *nu0 = xmalloc(sizeof(double) * N),
           *f0 = xmalloc(sizeof(double) * N);
    memset(rt, 0, sizeof(double) * N);
    for (int k = 0; k < nt; k++) {
        oracle_interp(s->n, rt + (long)k * N, s->Df, nu0);
        oracle_interp(s->n, src + (long)k * N, s->Df, f0);
        for (long p = 0; p < N; p++)
            rt[(long)(k + 1) * N + p] = nu0[p] + 0.5 * dt * (f0[p] + src[(long)(k + 1) * N + p]);
    }
    /* sources s^k = div(lam^k vt) of the incremental adjoint */
    double *sk = xmalloc(sizeof(double) * (nt + 1) * N), *lv = xmalloc(sizeof(double) * 3 * N);
    for (int k = 0; k <= nt; k++) {
        for (int j = 0; j < 3; j++)
            for (long p = 0; p < N; p++) lv[j * N + p] = lamg[(long)k * N + p] * vt[j * N + p];
        oracle_div(s->n, lv, sk + (long)k * N);
    }
    /* incremental adjoint lam~^nt..lam~^0 from lam~(1) = -rho~(1) */
    double *lam = xmalloc(sizeof(double) * (nt + 1) * N), *sX = xmalloc(sizeof(double) * N);
    for (long p = 0; p < N; p++) lam[(long)nt * N + p] = -rt[(long)nt * N + p];
    for (int k = nt; k > 0; k--) {
        oracle_interp(s->n, lam + (long)k * N, s->Da, nu0);
        oracle_interp(s->n, sk + (long)k * N, s->Da, sX);
        for (long p = 0; p < N; p++) {
            double cx = s->c ? s->c[p] : 0.0, cX = s->cX ? s->cX[p] : 0.0;
            double f00 = nu0[p] * cX + sX[p];
            double nus = nu0[p] + dt * f00;
            double fs = nus * cx + sk[(long)(k - 1) * N + p];
            lam[(long)(k - 1) * N + p] = nu0[p] + 0.5 * dt * (f00 + fs);
        }
    }
    /* b~ = sum_n w_n (lam~^n grad rho^n + lam^n grad rho~^n) */
    double *bt = xmalloc(sizeof(double) * 3 * N), *gt = xmalloc(sizeof(double) * 3 * N);
    accumulate_b(s, lam, bt);
    for (int k = 0; k <= nt; k++) {
        double w = trap_w(k, nt);
        oracle_grad(s->n, rt + (long)k * N, gt);
        for (int j = 0; j < 3; j++)
            for (long p = 0; p < N; p++) bt[j * N + p] += w * lamg[(long)k * N + p] * gt[j * N + p];
    }
    assemble(s->n, beta, s->iso, vt, bt, Hvt);
    free(src);
    free(rt);
    free(nu0);
    free(f0);
    free(sk);
    free(lv);
    free(lam);
    free(sX);
    free(bt);
    free(gt);
}

static int check_params(const oracle_params *P) {
    for (int j = 0; j < 3; j++)
        if (P->n[j] < 4) return 1;
    if (P->nt < 1 || !(P->beta > 0)) return 1;
    return 0;
}

/* exported: state solve; returns rho^nt (and the whole history if hist != NULL) */
int oracle_transport_forward(const oracle_params *P, const double *v, const double *rho0, double *rho1,
                             double *hist) {
    if (check_params(P)) return 1;
    long N = npts(P->n);
    double *Df = xmalloc(sizeof(double) * 3 * N), *h = xmalloc(sizeof(double) * (P->nt + 1) * N);
    oracle_backtrace(P->n, P->nt, v, +1.0, Df);
    oracle_state(P->n, P->nt, Df, rho0, h);
    memcpy(rho1, h + (long)P->nt * N, sizeof(double) * N);
    if (hist) memcpy(hist, h, sizeof(double) * (P->nt + 1) * N);
    free(Df);
    free(h);
    return 0;
}

/* exported: adjoint solve from lam(1) = lam1 back to lam(0) */
int oracle_transport_adjoint(const oracle_params *P, const double *v, const double *lam1, double *lam0) {
    if (check_params(P)) return 1;
    long N = npts(P->n);
    int nt = P->nt;
    double *Da = xmalloc(sizeof(double) * 3 * N), *h = xmalloc(sizeof(double) * (nt + 1) * N);
    double *c = NULL, *cX = NULL;
    oracle_backtrace(P->n, nt, v, -1.0, Da);
    if (!P->isochoric) {
        c = xmalloc(sizeof(double) * N);
        cX = xmalloc(sizeof(double) * N);
        oracle_div(P->n, v, c);
        oracle_interp(P->n, c, Da, cX);
    }
    oracle_adjoint(P->n, nt, Da, c, cX, lam1, h);
    memcpy(lam0, h, sizeof(double) * N);
    free(Da);
    free(h);
    free(c);
    free(cX);
    return 0;
}

/* exported: g, J, mismatch at v */
int oracle_gradient(const oracle_params *P, const double *rhoT, const double *rhoR, const double *v, double *g,
                    double *J, double *mismatch) {
    if (check_params(P)) return 1;
    oracle_state_t s;
    st_forward(&s, P->n, P->nt, P->isochoric, v, rhoT);
    st_complete(&s, v);
    double mis;
    double j = objective(&s, P->beta, v, rhoT, rhoR, &mis);
    gradient_from_state(&s, P->beta, v, rhoR, g, NULL);
    if (J) *J = j;
    if (mismatch) *mismatch = mis;
    st_free(&s);
    return 0;
}

/* exported: Gauss-Newton H(v) vt */
int oracle_hessian_matvec(const oracle_params *P, const double *rhoT, const double *v, const double *vt,
                          double *Hvt) {
    if (check_params(P)) return 1;
    oracle_state_t s;
    st_forward(&s, P->n, P->nt, P->isochoric, v, rhoT);
    st_complete(&s, v);
    hessian_from_state(&s, P->beta, vt, Hvt);
    st_free(&s);
    return 0;
}

/* exported: full Newton H(v) vt (needs rho_R for the adjoint history) */
int oracle_newton_matvec(const oracle_params *P, const double *rhoT, const double *rhoR, const double *v,
                         const double *vt, double *Hvt) {
    if (check_params(P)) return 1;
    oracle_state_t s;
    st_forward(&s, P->n, P->nt, P->isochoric, v, rhoT);
    st_complete(&s, v);
    long N = s.N;
    int nt = s.nt;
    double *lam = xmalloc(sizeof(double) * (nt + 1) * N), *lam1 = xmalloc(sizeof(double) * N);
    const double *r1 = s.rho + (long)nt * N;
    for (long p = 0; p < N; p++) lam1[p] = rhoR[p] - r1[p];
    oracle_adjoint(s.n, nt, s.Da, s.c, s.cX, lam1, lam);
    newton_from_state(&s, P->beta, lam, vt, Hvt);
    free(lam);
    free(lam1);
    st_free(&s);
    return 0;
}

/* exported: objective only (plan + state solve) */
int oracle_objective(const oracle_params *P, const double *rhoT, const double *rhoR, const double *v, double *J,
                     double *mismatch) {
    if (check_params(P)) return 1;
    oracle_state_t s;
    st_forward(&s, P->n, P->nt, P->isochoric, v, rhoT);
    *J = objective(&s, P->beta, v, rhoT, rhoR, mismatch);
    st_free(&s);
    return 0;
}

/* exported: u = y1 - x by transporting y like the state (eq. (1)):
 * u^{n+1} = u^n(X) + h D, u^0 = 0; then det(I + grad u) with min and max */
int oracle_deformation(const oracle_params *P, const double *v, double *u, double *det, double *detmin,
                       double *detmax) {
    if (check_params(P)) return 1;
    const int *n = P->n;
    long N = npts(n);
    int nt = P->nt;
    double *Df = xmalloc(sizeof(double) * 3 * N), *tmp = xmalloc(sizeof(double) * N);
    oracle_backtrace(n, nt, v, +1.0, Df);
    memset(u, 0, sizeof(double) * 3 * N);
    for (int k = 0; k < nt; k++)
        for (int j = 0; j < 3; j++) {
            double h = TWO_PI / n[j];
            oracle_interp(n, u + j * N, Df, tmp);
            for (long p = 0; p < N; p++) u[j * N + p] = tmp[p] + h * Df[j * N + p];
        }
    double *du = xmalloc(sizeof(double) * 9 * N); /* du[(a*3+b)N] = d_b u_a */
    for (int a = 0; a < 3; a++)
        for (int b = 0; b < 3; b++) oracle_deriv(n, b, u + a * N, du + (a * 3 + b) * N);
    double mn = INFINITY, mx = -INFINITY;
    for (long p = 0; p < N; p++) {
        double F[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) F[a][b] = (a == b ? 1.0 : 0.0) + du[(a * 3 + b) * N + p];
        double d = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) - F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                   F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
        if (det) det[p] = d;
        if (d < mn) mn = d;
        if (d > mx) mx = d;
    }
    *detmin = mn;
    *detmax = mx;
    free(Df);
    free(tmp);
    free(du);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gauss-Newton-Krylov solver (section III-A)                           */
/* ------------------------------------------------------------------ */

#define ORACLE_MAXIT 512

typedef struct {
    int32_t status;      /* 0 ok, 6 line search failed */
    int32_t n_iter;      /* accepted Newton steps recorded below */
    int32_t matvecs, gradients, objectives, stop_reason; /* 0 gtol, 1 mismatch, 2 max_newton */
    double J[ORACLE_MAXIT], mismatch[ORACLE_MAXIT], grel[ORACLE_MAXIT], alpha[ORACLE_MAXIT], beta[ORACLE_MAXIT];
    int32_t pcg_iters[ORACLE_MAXIT], ls_trials[ORACLE_MAXIT];
    double final_J, final_mismatch, final_grel;
    double final_beta;   /* beta of the last continuation level worked on */
    double final_gref;   /* that level's gradient reference */
    int32_t negative_curvature; /* PCG runs ended by <p, H p> <= 0 */
    int32_t descent_fallbacks;  /* Newton steps whose PCG step was no descent direction (replaced by -M g) */
} oracle_report;

static double norm3(const int *n, const double *x) { return sqrt(inner(n, 3, x, x)); }

int oracle_solve(const oracle_params *P, const double *rhoT, const double *rhoR, double *v, oracle_report *rep) {
    const int progress = getenv("ORACLE_PROGRESS") != NULL;
    if (check_params(P)) return 1;
    memset(rep, 0, sizeof(*rep));
    const int *n = P->n;
    long N = npts(n), N3 = 3 * N;
    double *g = xmalloc(sizeof(double) * N3), *s = xmalloc(sizeof(double) * N3), *r = xmalloc(sizeof(double) * N3);
    double *z = xmalloc(sizeof(double) * N3), *pp = xmalloc(sizeof(double) * N3), *q = xmalloc(sizeof(double) * N3);
    double *vtrial = xmalloc(sizeof(double) * N3);
    /* adjoint history of the current gradient (full Newton only) */
    double *lamg = P->hessian ? xmalloc(sizeof(double) * (P->nt + 1) * N) : NULL;

    if (P->isochoric) {
        oracle_leray(n, v, vtrial);
        memcpy(v, vtrial, sizeof(double) * N3);
    }
    double beta = P->beta;
    double beta_final = P->beta_final > 0 ? P->beta_final : P->beta;
    double factor = (P->beta_factor > 0 && P->beta_factor < 1) ? P->beta_factor : 0.1;
    int done = 0, it = 0, first_level = 1;
    double J = 0, mis = 0, gnorm = 0, g0 = 0;
    while (!done) {
        oracle_state_t st;
        st_forward(&st, n, P->nt, P->isochoric, v, rhoT);
        st_complete(&st, v);
        J = objective(&st, beta, v, rhoT, rhoR, &mis);
        gradient_from_state(&st, beta, v, rhoR, g, lamg);
        rep->gradients++;
        gnorm = norm3(n, g);
        g0 = (first_level && P->gref_first > 0) ? P->gref_first : gnorm;
        first_level = 0;
        rep->stop_reason = 2;
        const double ref = P->gnorm_ref > 0 ? P->gnorm_ref : g0;
        const double tol = (P->gtol_level > 0 && beta > beta_final * (1 + 1e-12)) ? P->gtol_level : P->gtol;
        for (int k = 0; k < P->max_newton; k++) {
            if (gnorm <= tol * ref) {
                rep->stop_reason = 0;
                break;
            }
            if (P->mismatch_tol > 0 && mis <= P->mismatch_tol) {
                rep->stop_reason = 1;
                break;
            }
            double ratio = ref > 0 ? gnorm / ref : 0.0;
            double eta = P->forcing == 1 ? sqrt(ratio) : ratio;
            if (eta > 0.5) eta = 0.5;
            /* truncated PCG on H s = -g */
            memset(s, 0, sizeof(double) * N3);
            for (long i = 0; i < N3; i++) r[i] = -g[i];
            oracle_precond(n, beta, P->isochoric, r, z);
            memcpy(pp, z, sizeof(double) * N3);
            double rz = inner(n, 3, r, z);
            int iters = 0;
            for (int i = 0; i < P->max_pcg; i++) {
                if (P->hessian) newton_from_state(&st, beta, lamg, pp, q);
                else hessian_from_state(&st, beta, pp, q);
                rep->matvecs++;
                iters = i + 1;
                if (progress && iters % 10 == 0) fprintf(stderr, "[oracle]   pcg iteration %d\n", iters);
                double kappa = inner(n, 3, pp, q);
                if (kappa <= 0) {
                    rep->negative_curvature++;
                    if (i == 0) memcpy(s, z, sizeof(double) * N3);
                    break;
                }
                double a = rz / kappa;
                for (long t = 0; t < N3; t++) {
                    s[t] += a * pp[t];
                    r[t] -= a * q[t];
                }
                if (norm3(n, r) <= eta * gnorm) break;
                oracle_precond(n, beta, P->isochoric, r, z);
                double rz1 = inner(n, 3, r, z);
                double bb = rz1 / rz;
                for (long t = 0; t < N3; t++) pp[t] = z[t] + bb * pp[t];
                rz = rz1;
            }
            /* Armijo backtracking on J(v + alpha s); a step that is not a
             * descent direction (possible with a truncated or indefinite
             * solve) is replaced by the preconditioned steepest descent
             * direction -M g */
            double alpha = 1.0, d = inner(n, 3, g, s);
            if (!(d < 0)) {
                for (long t = 0; t < N3; t++) r[t] = -g[t];
                oracle_precond(n, beta, P->isochoric, r, s);
                d = inner(n, 3, g, s);
                rep->descent_fallbacks++;
            }
            int accepted = 0, trials = 0;
            oracle_state_t tr;
            memset(&tr, 0, sizeof(tr));
            double Jt = 0, mist = 0;
            for (int l = 0; l < P->max_ls; l++) {
                trials++;
                for (long t = 0; t < N3; t++) vtrial[t] = v[t] + alpha * s[t];
                st_free(&tr);
                st_forward(&tr, n, P->nt, P->isochoric, vtrial, rhoT);
                Jt = objective(&tr, beta, vtrial, rhoT, rhoR, &mist);
                rep->objectives++;
                if (Jt <= J + P->armijo_c1 * alpha * d) {
                    accepted = 1;
                    break;
                }
                alpha *= 0.5;
            }
            if (!accepted) {
                st_free(&tr);
                st_free(&st);
                rep->status = 6;
                goto out;
            }
            memcpy(v, vtrial, sizeof(double) * N3);
            st_free(&st);
            st = tr;
            st_complete(&st, v);
            J = Jt;
            mis = mist;
            gradient_from_state(&st, beta, v, rhoR, g, lamg);
            rep->gradients++;
            gnorm = norm3(n, g);
            if (it < ORACLE_MAXIT) {
                rep->J[it] = J;
                rep->mismatch[it] = mis;
                rep->grel[it] = g0 > 0 ? gnorm / g0 : 0;
                rep->alpha[it] = alpha;
                rep->beta[it] = beta;
                rep->pcg_iters[it] = iters;
                rep->ls_trials[it] = trials;
            }
            /* a line per accepted step on stderr when ORACLE_PROGRESS is set,
             * so that long runs show that they advance (no arithmetic here) */
            if (progress)
                fprintf(stderr, "[oracle] step %d: beta %.1e, J %.6e, mismatch %.6f, |g|/|g0| %.3e, pcg %d\n", it,
                        beta, J, mis, g0 > 0 ? gnorm / g0 : 0.0, iters);
            it++;
            rep->stop_reason = 2;
        }
        /* the loop may also end after its last step without a test */
        if (rep->stop_reason == 2) {
            if (gnorm <= tol * ref) rep->stop_reason = 0;
            if (P->mismatch_tol > 0 && mis <= P->mismatch_tol) rep->stop_reason = 1;
        }
        st_free(&st);
        if (rep->stop_reason == 1 || beta <= beta_final * (1 + 1e-12)) done = 1;
        else {
            beta *= factor;
            if (beta < beta_final) beta = beta_final;
        }
    }
out:
    rep->n_iter = it;
    rep->final_J = J;
    rep->final_mismatch = mis;
    rep->final_grel = g0 > 0 ? gnorm / g0 : 0;
    rep->final_beta = beta;
    rep->final_gref = g0;
    free(g);
    free(s);
    free(r);
    free(z);
    free(pp);
    free(q);
    free(vtrial);
    free(lamg);
    return rep->status;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}
