/* The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
 * (host code, gcc) and driven through its entry points on small grids: FFT,
 * derivatives, Leray, resampling, interpolation and its transpose,
 * backtrace, transports, gradient, Gauss-Newton and full Newton matvecs,
 * the deformation map and two solves (isochoric, and a grid whose axes are
 * 2 3^b 5^c). Any out-of-bounds access, leak or undefined operation aborts the
 * run with a report; on success the line "ok <checksum>" is printed. */
#include "../../oracle/oracle.c"

static double checksum(const double *x, long n) {
    double s = 0;
    for (long i = 0; i < n; i++) s += x[i] * (double)((i % 7) + 1);
    return s;
}

static void fields(const int n[3], double *rhoT, double *v) {
    const long N = (long)n[0] * n[1] * n[2];
    for (int i = 0; i < n[0]; i++)
        for (int j = 0; j < n[1]; j++)
            for (int k = 0; k < n[2]; k++) {
                const double x1 = TWO_PI * i / n[0], x2 = TWO_PI * j / n[1], x3 = TWO_PI * k / n[2];
                const long p = ((long)i * n[1] + j) * n[2] + k;
                rhoT[p] = (sin(x1) * sin(x1) + sin(x2) * sin(x2) + sin(x3) * sin(x3)) / 3;
                v[p] = 0.5 * sin(x3) * cos(x2) * sin(x2);
                v[N + p] = 0.5 * sin(x1) * cos(x3) * sin(x3);
                v[2 * N + p] = 0.5 * sin(x2) * cos(x1) * sin(x1);
            }
}

static double run(const int n[3], int isochoric, int hessian) {
    const long N = (long)n[0] * n[1] * n[2];
    double *rhoT = calloc(N, 8), *rhoR = calloc(N, 8), *v = calloc(3 * N, 8), *g = calloc(3 * N, 8);
    double *w = calloc(3 * N, 8), *D = calloc(3 * N, 8), *out = calloc(3 * N, 8), *det = calloc(N, 8);
    double *cin = calloc(2 * N, 8), *spec = calloc(2 * N, 8), *lam = calloc(N, 8), *small = calloc(3 * N, 8);
    fields(n, rhoT, v);
    oracle_params P;
    memset(&P, 0, sizeof(P));
    for (int j = 0; j < 3; j++) P.n[j] = n[j];
    P.nt = 3;
    P.beta = P.beta_final = 1e-2;
    P.beta_factor = 0.1;
    P.isochoric = isochoric;
    P.gtol = 1e-2;
    P.max_newton = 2;
    P.max_pcg = 10;
    P.max_ls = 5;
    P.hessian = hessian;
    P.armijo_c1 = 1e-4;
    double s = 0, J = 0, mis = 0, dmin = 0, dmax = 0;
    for (long i = 0; i < N; i++) cin[2 * i] = rhoT[i], cin[2 * i + 1] = v[i];
    oracle_fft3(n, cin, spec, -1);
    s += checksum(spec, 2 * N);
    oracle_deriv(n, 0, rhoT, out);
    oracle_grad(n, rhoT, out);
    oracle_div(n, v, lam);
    oracle_leray(n, v, out);
    oracle_precond(n, 1e-2, isochoric, v, out);
    const int m[3] = {n[0] / 2, n[1] / 2, n[2] / 2};
    oracle_resample(n, m, 3, v, small);
    s += checksum(out, 3 * N) + checksum(small, 3 * (N / 8));
    oracle_backtrace(n, P.nt, v, 1.0, D);
    oracle_interp(n, rhoT, D, out);
    oracle_interp_transpose(n, rhoT, D, w);
    s += checksum(out, N) + checksum(w, N);
    /* displacements of several periods either way: the periodic wrap of the stencil */
    for (int j = 0; j < 3; j++)
        for (long p = 0; p < N; p++) D[j * N + p] = (4.0 * ((p * 37 + j * 11) % 101) / 100.0 - 2.0) * n[j] - 0.5;
    oracle_interp(n, rhoT, D, out);
    oracle_interp_transpose(n, rhoT, D, w);
    for (int which = 0; which < 4; which++) {
        oracle_even_op(n, 3, which, 0.3, v, small);
        s += checksum(small, 3 * N);
    }
    s += checksum(out, N) + checksum(w, N) + oracle_regulariser(n, 1e-2, v);
    if (oracle_transport_forward(&P, v, rhoT, rhoR, NULL)) return NAN;
    if (oracle_transport_adjoint(&P, v, rhoR, lam)) return NAN;
    if (oracle_gradient(&P, rhoT, rhoR, v, g, &J, &mis)) return NAN;
    if (oracle_hessian_matvec(&P, rhoT, v, g, out)) return NAN;
    if (oracle_newton_matvec(&P, rhoT, rhoR, v, g, w)) return NAN;
    if (oracle_deformation(&P, v, out, det, &dmin, &dmax)) return NAN;
    double J2 = 0, mis2 = 0;
    if (oracle_objective(&P, rhoT, rhoR, v, &J2, &mis2)) return NAN;
    s += J + mis + J2 + mis2 + checksum(out, 3 * N) + checksum(w, 3 * N) + dmin + dmax;
    /* a solve from half the velocity that produced rho_R */
    for (long i = 0; i < 3 * N; i++) w[i] = 0.5 * v[i];
    oracle_report rep;
    if (oracle_solve(&P, rhoT, rhoR, w, &rep)) return NAN;
    s += rep.final_J + rep.matvecs;
    free(rhoT); free(rhoR); free(v); free(g); free(w); free(D); free(out); free(det); free(cin); free(spec); free(lam);
    free(small);
    return s;
}

int main(void) {
    const int a[3] = {8, 12, 16}, b[3] = {10, 12, 6};
    const double s = run(a, 0, 1) + run(a, 1, 0) + run(b, 0, 0);
    if (!isfinite(s)) {
        printf("failed\n");
        return 1;
    }
    printf("ok %.6e\n", s);
    return 0;
}
