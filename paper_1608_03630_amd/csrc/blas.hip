// Vector updates and double-precision reductions for the Newton-Krylov
// driver (section III-A of the paper: matrix-free PCG and Armijo line search
// over grid vectors). Reductions are deterministic: a fixed grid of blocks
// reduces by wavefront shuffles (64 lanes) and a fixed-order block sum, and
// one block adds the per-block partials in index order, so repeated runs give
// bitwise identical scalars.
#include "common.hpp"

namespace regk {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}
__device__ __forceinline__ double wave_min(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
    return v;
}
__device__ __forceinline__ double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
    return v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_dot_partials(const T *__restrict__ a, const T *__restrict__ b, long n,
                                                           int mode, double *__restrict__ partials) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
        const double x = (double)a[i];
        if (mode == 0) acc += x * (double)b[i];
        else if (mode == 1) {
            const double d = x - (double)b[i];
            acc += d * d;
        } else acc += x * x;
    }
    acc = wave_sum(acc);
    __shared__ double ws[kThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; i++) t += ws[i];
        partials[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kThreads) void k_finalize(const double *__restrict__ partials, int nparts, double scale,
                                                       double *__restrict__ out) {
    // each thread sums a strided subset in order, then a fixed tree
    double acc = 0.0;
    for (int i = threadIdx.x; i < nparts; i += kThreads) acc += partials[i];
    acc = wave_sum(acc);
    __shared__ double ws[kThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; i++) t += ws[i];
        out[0] = scale * t;
    }
}

// det of F = I + grad u with F_ab = delta_ab + d_b u_a, du[(a*3+b)*n + i]
template <typename T>
__global__ __launch_bounds__(kThreads) void k_det_partials(const T *__restrict__ du, long n,
                                                           double *__restrict__ pmin, double *__restrict__ pmax,
                                                           T *__restrict__ det_out) {
    double mn = INFINITY, mx = -INFINITY;
    for (long i = (long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long)gridDim.x * kThreads) {
        double F[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) F[a][b] = (a == b ? 1.0 : 0.0) + (double)du[(a * 3 + b) * n + i];
        const double d = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                         F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                         F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
        if (det_out) det_out[i] = (T)d;
        mn = fmin(mn, d);
        mx = fmax(mx, d);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    __shared__ double wmn[kThreads / 64], wmx[kThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        wmn[threadIdx.x >> 6] = mn;
        wmx[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < kThreads / 64; i++) {
            mn = fmin(mn, wmn[i]);
            mx = fmax(mx, wmx[i]);
        }
        mn = fmin(mn, wmn[0]);
        mx = fmax(mx, wmx[0]);
        pmin[blockIdx.x] = mn;
        pmax[blockIdx.x] = mx;
    }
}

__global__ __launch_bounds__(kThreads) void k_finalize_minmax(const double *__restrict__ pmin,
                                                              const double *__restrict__ pmax, int nparts,
                                                              double *__restrict__ out2) {
    double mn = INFINITY, mx = -INFINITY;
    for (int i = threadIdx.x; i < nparts; i += kThreads) {
        mn = fmin(mn, pmin[i]);
        mx = fmax(mx, pmax[i]);
    }
    mn = wave_min(mn);
    mx = wave_max(mx);
    __shared__ double wmn[kThreads / 64], wmx[kThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        wmn[threadIdx.x >> 6] = mn;
        wmx[threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 0; i < kThreads / 64; i++) {
            mn = fmin(mn, wmn[i]);
            mx = fmax(mx, wmx[i]);
        }
        out2[0] = mn;
        out2[1] = mx;
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_fill(long n, T v, T *__restrict__ y) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = v;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_copy(long n, const T *__restrict__ x, T *__restrict__ y) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = x[i];
}

template <typename Ti, typename To>
__global__ __launch_bounds__(kThreads) void k_convert(long n, const Ti *__restrict__ x, To *__restrict__ y) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = To(x[i]);
}

// Streaming kernels of the full Newton Hessian matvec (eqs. (5a)-(5e) with
// the lam terms of section II-B).

// out_j = lam * vt_j for the three components
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale_vec(long n, const T *__restrict__ lam, const T *__restrict__ vt,
                                                        T *__restrict__ out) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const T l = lam[i];
    out[i] = l * vt[i];
    out[n + i] = l * vt[n + i];
    out[2 * n + i] = l * vt[2 * n + i];
}

// q += cs * (vt . grad)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_add_vdotgrad(long n, const T *__restrict__ vt, const T *__restrict__ g,
                                                           T *__restrict__ q, T cs) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    q[i] += cs * (vt[i] * g[i] + vt[n + i] * g[n + i] + vt[2 * n + i] * g[2 * n + i]);
}

// The source part of one incremental-adjoint step with f = nu c + s (eq. (7)
// expanded; the nu part, nu(X) gam, is already in out):
// out += s(X) dt/2 (1 + dt c) + dt/2 s_next, c = div v (null: 0)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_newton_source(long n, const T *__restrict__ sX,
                                                            const T *__restrict__ s_next, const T *__restrict__ c,
                                                            T dt, T *__restrict__ out) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const T h = T(0.5) * dt;
    const T a = c ? h * (T(1) + dt * c[i]) : h;
    out[i] += a * sX[i] + h * s_next[i];
}

// b_j += w lam g_j for the three components
template <typename T>
__global__ __launch_bounds__(kThreads) void k_b_axpy(long n, T w, const T *__restrict__ lam, const T *__restrict__ g,
                                                     T *__restrict__ b) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const T s = w * lam[i];
    b[i] += s * g[i];
    b[n + i] += s * g[n + i];
    b[2 * n + i] += s * g[2 * n + i];
}

// y = a x
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scale(long n, T a, const T *__restrict__ x, T *__restrict__ y) {
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) y[i] = a * x[i];
}

// Zero padding of an m-sized image into the centre of the n-sized grid
// (offset o = (n - m) / 2 per axis), zeros elsewhere; and the inverse crop.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pad(Grid g, int m1, int m2, int m3, int o1, int o2, int o3,
                                                  const T *__restrict__ img, T *__restrict__ out) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= g.N()) return;
    const int i3 = (int)(p % g.n3), i2 = (int)((p / g.n3) % g.n2), i1 = (int)(p / ((long)g.n2 * g.n3));
    const int a1 = i1 - o1, a2 = i2 - o2, a3 = i3 - o3;
    const bool in = a1 >= 0 && a1 < m1 && a2 >= 0 && a2 < m2 && a3 >= 0 && a3 < m3;
    out[p] = in ? img[((long)a1 * m2 + a2) * m3 + a3] : T(0);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_crop(Grid g, int m1, int m2, int m3, int o1, int o2, int o3,
                                                   const T *__restrict__ f, T *__restrict__ out) {
    const long q = (long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= (long)m1 * m2 * m3) return;
    const int a3 = (int)(q % m3), a2 = (int)((q / m3) % m2), a1 = (int)(q / ((long)m2 * m3));
    out[q] = f[((long)(a1 + o1) * g.n2 + (a2 + o2)) * g.n3 + (a3 + o3)];
}

inline unsigned nb(long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

template <typename T>
hipError_t launch_pad(const Grid &g, const int m[3], const T *img, T *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pad<T>, dim3(nb(g.N())), dim3(kThreads), 0, s, g, m[0], m[1], m[2], (g.n1 - m[0]) / 2,
                       (g.n2 - m[1]) / 2, (g.n3 - m[2]) / 2, img, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_crop(const Grid &g, const int m[3], const T *f, T *out, hipStream_t s) {
    hipLaunchKernelGGL(k_crop<T>, dim3(nb((long)m[0] * m[1] * m[2])), dim3(kThreads), 0, s, g, m[0], m[1], m[2],
                       (g.n1 - m[0]) / 2, (g.n2 - m[1]) / 2, (g.n3 - m[2]) / 2, f, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale_vec(long n, const T *lam, const T *vt, T *out, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_vec<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, lam, vt, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_add_vdotgrad(long n, const T *vt, const T *g, T *q, double cs, hipStream_t s) {
    hipLaunchKernelGGL(k_add_vdotgrad<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, vt, g, q, T(cs));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_newton_source(long n, const T *sX, const T *s_next, const T *c, double dt, T *out, hipStream_t s) {
    hipLaunchKernelGGL(k_newton_source<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, sX, s_next, c, T(dt), out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_b_axpy(long n, double w, const T *lam, const T *g, T *b, hipStream_t s) {
    hipLaunchKernelGGL(k_b_axpy<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, T(w), lam, g, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_scale(long n, double a, const T *x, T *y, hipStream_t s) {
    hipLaunchKernelGGL(k_scale<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, T(a), x, y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dot_partials(const T *a, const T *b, long n, int mode, double *partials, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_partials<T>, dim3(RED_BLOCKS), dim3(kThreads), 0, s, a, b, n, mode, partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *partials, int nparts, double scale, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kThreads), 0, s, partials, nparts, scale, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_det_partials(const T *du, long n, double *pmin, double *pmax, T *det_out, hipStream_t s) {
    hipLaunchKernelGGL(k_det_partials<T>, dim3(RED_BLOCKS), dim3(kThreads), 0, s, du, n, pmin, pmax, det_out);
    return hipGetLastError();
}

hipError_t launch_finalize_minmax(const double *pmin, const double *pmax, int nparts, double *out2, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_minmax, dim3(1), dim3(kThreads), 0, s, pmin, pmax, nparts, out2);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(long n, double val, T *y, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, T(val), y);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_copy(long n, const T *x, T *y, hipStream_t s) {
    hipLaunchKernelGGL(k_copy<T>, dim3(nb(n)), dim3(kThreads), 0, s, n, x, y);
    return hipGetLastError();
}

template <typename Ti, typename To>
hipError_t launch_convert(long n, const Ti *x, To *y, hipStream_t s) {
    hipLaunchKernelGGL((k_convert<Ti, To>), dim3(nb(n)), dim3(kThreads), 0, s, n, x, y);
    return hipGetLastError();
}
template hipError_t launch_convert<double, float>(long, const double *, float *, hipStream_t);
template hipError_t launch_convert<float, double>(long, const float *, double *, hipStream_t);

#define REGK_BLAS_INST(T)                                                                                          \
    template hipError_t launch_dot_partials<T>(const T *, const T *, long, int, double *, hipStream_t);            \
    template hipError_t launch_det_partials<T>(const T *, long, double *, double *, T *, hipStream_t);             \
    template hipError_t launch_fill<T>(long, double, T *, hipStream_t);                                            \
    template hipError_t launch_copy<T>(long, const T *, T *, hipStream_t);                                          \
    template hipError_t launch_scale_vec<T>(long, const T *, const T *, T *, hipStream_t);                         \
    template hipError_t launch_add_vdotgrad<T>(long, const T *, const T *, T *, double, hipStream_t);             \
    template hipError_t launch_newton_source<T>(long, const T *, const T *, const T *, double, T *, hipStream_t);  \
    template hipError_t launch_b_axpy<T>(long, double, const T *, const T *, T *, hipStream_t);                    \
    template hipError_t launch_scale<T>(long, double, const T *, T *, hipStream_t);                                \
    template hipError_t launch_pad<T>(const Grid &, const int *, const T *, T *, hipStream_t);                     \
    template hipError_t launch_crop<T>(const Grid &, const int *, const T *, T *, hipStream_t);

REGK_BLAS_INST(float)
REGK_BLAS_INST(double)

}  // namespace regk
