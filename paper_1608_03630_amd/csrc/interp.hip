// Semi-Lagrangian transport kernels for gfx950: periodic tricubic Lagrange
// interpolation at departure points (sections III-B2 and III-C2 of the
// paper), the RK2 characteristic backtrace (eq. (6)) and the fused time-step
// kernels of the state, adjoint, incremental-state and incremental-adjoint
// solves (eq. (7)) and of the deformation map (eq. (1)).
//
// One thread per grid point, which gathers its 4x4x4 stencil and evaluates it
// separably (16 rows of 4 along x3, then 4 planes along x2, then x1): 64 FMA
// instead of the 64-term product sum, and every output point is written by
// exactly one thread (a race-free gather). Blocks are remapped so that each
// XCD (8 per MI355X, one L2 each) receives a contiguous slab of the grid,
// which keeps the stencil halos of neighbouring blocks in the same L2.
#include "common.hpp"

namespace regk {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;

// Hardware dispatches consecutive workgroups round-robin over the XCDs; map
// them back so that XCD x works on the x-th contiguous share of the grid.
__device__ __forceinline__ long xcd_block() {
    const unsigned b = blockIdx.x, nb = gridDim.x;
    const unsigned q = nb / kXcds, r = nb % kXcds;
    const unsigned x = b % kXcds, t = b / kXcds;
    const unsigned base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return (long)(base + t);
}

__device__ __forceinline__ int wrap_idx(int m, int n) {
    const int r = m % n;
    return r < 0 ? r + n : r;
}

template <typename T> __device__ __forceinline__ T flo(T x);
template <> __device__ __forceinline__ float flo<float>(float x) { return floorf(x); }
template <> __device__ __forceinline__ double flo<double>(double x) { return floor(x); }

// cubic Lagrange basis on the nodes -1, 0, 1, 2 at t in [0, 1)
template <typename T>
__device__ __forceinline__ void lagrange4(T t, T w[4]) {
    const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
    w[0] = -t * tm1 * tm2 * T(1.0 / 6.0);
    w[1] = tp1 * tm1 * tm2 * T(0.5);
    w[2] = -tp1 * t * tm2 * T(0.5);
    w[3] = tp1 * t * tm1 * T(1.0 / 6.0);
}

// The stencil of one departure point: wrapped element offsets per axis and
// the per-axis weights.
template <typename T>
struct Stencil {
    int o1[4], o2[4], o3[4];
    T w1[4], w2[4], w3[4];
};

template <typename T>
__device__ __forceinline__ void axis_stencil(int i, T d, int n, int stride, int o[4], T w[4]) {
    const T fl = flo(d);
    const T t = d - fl;  // exact
    // clamp before the conversion (NaN maps to the lower bound); the modulo
    // then keeps every stencil index inside [0, n)
    const T flc = fmin(fmax(fl, T(-1e9)), T(1e9));
    const int base = wrap_idx(i + (int)flc - 1, n);  // |i + flc| < 2^31
    int x = base;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        o[a] = x * stride;
        x = (x + 1 == n) ? 0 : x + 1;
    }
    lagrange4(t, w);
}

template <typename T>
__device__ __forceinline__ void make_stencil(const Grid &g, int i1, int i2, int i3, T d1, T d2, T d3,
                                             Stencil<T> &st) {
    axis_stencil(i1, d1, g.n1, g.n2 * g.n3, st.o1, st.w1);
    axis_stencil(i2, d2, g.n2, g.n3, st.o2, st.w2);
    axis_stencil(i3, d3, g.n3, 1, st.o3, st.w3);
}

template <typename T>
__device__ __forceinline__ T apply(const T *__restrict__ f, const Stencil<T> &st) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; a++) {
        T pa = T(0);
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const T *row = f + st.o1[a] + st.o2[b];
            const T r = st.w3[0] * row[st.o3[0]] + st.w3[1] * row[st.o3[1]] + st.w3[2] * row[st.o3[2]] +
                        st.w3[3] * row[st.o3[3]];
            pa += st.w2[b] * r;
        }
        acc += st.w1[a] * pa;
    }
    return acc;
}

struct PointIdx {
    long p;
    int i1, i2, i3;
};

// grids hold fewer than 2^31 points, so 32-bit index arithmetic suffices
__device__ __forceinline__ bool point_of(const Grid &g, PointIdx &pi) {
    const long p = xcd_block() * kThreads + threadIdx.x;
    if (p >= g.N()) return false;
    pi.p = p;
    const unsigned up = (unsigned)p, n3 = (unsigned)g.n3, n2 = (unsigned)g.n2;
    const unsigned r = up / n3;
    pi.i3 = (int)(up - r * n3);
    pi.i2 = (int)(r % n2);
    pi.i1 = (int)(r / n2);
    return true;
}

// ------------------------------------------------------------------ kernels

template <typename T>
__global__ __launch_bounds__(kThreads) void k_interp(Grid g, const T *__restrict__ f, const T *__restrict__ D,
                                                     T *__restrict__ out) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N();
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, D[pi.p], D[N + pi.p], D[2 * N + pi.p], st);
    out[pi.p] = apply(f, st);
}

// Departure points of sign*v, per axis with c = -sign*dt:
// D*_j = c v_j / h_j, then D_j = c (v_j(x) + v_j(X*)) / (2 h_j).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_backtrace(Grid g, const T *__restrict__ v, T c, T ih1, T ih2, T ih3,
                                                        T *__restrict__ D) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N();
    const T v1 = v[pi.p], v2 = v[N + pi.p], v3 = v[2 * N + pi.p];
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, c * v1 * ih1, c * v2 * ih2, c * v3 * ih3, st);
    const T w1 = apply(v, st), w2 = apply(v + N, st), w3 = apply(v + 2 * N, st);
    const T hc = T(0.5) * c;
    D[pi.p] = hc * (v1 + w1) * ih1;
    D[N + pi.p] = hc * (v2 + w2) * ih2;
    D[2 * N + pi.p] = hc * (v3 + w3) * ih3;
}

// One backward (tau) step of d_tau nu + (-v).grad nu = nu c with eq. (7):
// nu0 = nu(X), f0 = nu0 c(X), nu* = nu0 + dt f0, f* = nu* c(x),
// nu_new = nu0 + dt/2 (f0 + f*); then b += wn nu_new grad.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_step(Grid g, const T *__restrict__ lam_in,
                                                           const T *__restrict__ Da, const T *__restrict__ c,
                                                           const T *__restrict__ cX, const T *__restrict__ grad,
                                                           T *__restrict__ b, T *__restrict__ lam_out, T dt, T wn) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N(), p = pi.p;
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, Da[p], Da[N + p], Da[2 * N + p], st);
    T lam = apply(lam_in, st);
    if (c) {
        const T f0 = lam * cX[p];
        const T nus = lam + dt * f0;
        const T fs = nus * c[p];
        lam = lam + T(0.5) * dt * (f0 + fs);
    }
    if (lam_out) lam_out[p] = lam;
    if (b) {
        const T s = wn * lam;
        b[p] += s * grad[p];
        b[N + p] += s * grad[N + p];
        b[2 * N + p] += s * grad[2 * N + p];
    }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_init(long N, const T *__restrict__ rhoR,
                                                           const T *__restrict__ rho1, const T *__restrict__ grad,
                                                           T *__restrict__ lam, T *__restrict__ b, T w) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    const T l = rhoR[p] - rho1[p];
    lam[p] = l;
    if (b) {
        const T s = w * l;
        b[p] = s * grad[p];
        b[N + p] = s * grad[N + p];
        b[2 * N + p] = s * grad[2 * N + p];
    }
}

// q_out = q_in(X) + cs * (vt . grad rho^{n+1}); the last step writes
// lam~ = -(that) and starts b~ = w lam~ grad rho^{nt}.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_incstate_step(Grid g, const T *__restrict__ q_in,
                                                            const T *__restrict__ Df, const T *__restrict__ vt,
                                                            const T *__restrict__ grad, T *__restrict__ q_out, T cs,
                                                            int last, T *__restrict__ b, T w) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N(), p = pi.p;
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, Df[p], Df[N + p], Df[2 * N + p], st);
    const T g1 = grad[p], g2 = grad[N + p], g3 = grad[2 * N + p];
    const T s = vt[p] * g1 + vt[N + p] * g2 + vt[2 * N + p] * g3;
    T q = apply(q_in, st) + cs * s;
    if (last) {
        q = -q;
        const T ws = w * q;
        b[p] = ws * g1;
        b[N + p] = ws * g2;
        b[2 * N + p] = ws * g3;
    }
    q_out[p] = q;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_incstate_init(long N, const T *__restrict__ vt,
                                                            const T *__restrict__ grad, T *__restrict__ q, T cs) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    q[p] = cs * (vt[p] * grad[p] + vt[N + p] * grad[N + p] + vt[2 * N + p] * grad[2 * N + p]);
}

// u^{n+1}_j = u^n_j(X) + h_j D_j for the three components
template <typename T>
__global__ __launch_bounds__(kThreads) void k_deform_step(Grid g, const T *__restrict__ u_in,
                                                          const T *__restrict__ Df, T *__restrict__ u_out, T h1, T h2,
                                                          T h3) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N(), p = pi.p;
    const T d1 = Df[p], d2 = Df[N + p], d3 = Df[2 * N + p];
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, d1, d2, d3, st);
    u_out[p] = apply(u_in, st) + h1 * d1;
    u_out[N + p] = apply(u_in + N, st) + h2 * d2;
    u_out[2 * N + p] = apply(u_in + 2 * N, st) + h3 * d3;
}

inline unsigned nblocks(long N) { return (unsigned)((N + kThreads - 1) / kThreads); }

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T>
hipError_t launch_interp(const Grid &g, const T *f, const T *D, T *out, hipStream_t s) {
    hipLaunchKernelGGL(k_interp<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, f, D, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backtrace(const Grid &g, const T *v, double sign_dt, T *D, hipStream_t s) {
    const double pi2 = 6.283185307179586476925286766559;
    hipLaunchKernelGGL(k_backtrace<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, v, T(-sign_dt),
                       T(g.n1 / pi2), T(g.n2 / pi2), T(g.n3 / pi2), D);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_step(const Grid &g, const T *lam_in, const T *Da, const T *c, const T *cX, const T *grad,
                               T *b, T *lam_out, double dt, double wn, hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_step<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, lam_in, Da, c, cX, grad, b,
                       lam_out, T(dt), T(wn));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_init(const Grid &g, const T *rhoR, const T *rho1, const T *grad, T *lam, T *b, double w,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_init<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g.N(), rhoR, rho1, grad, lam,
                       b, T(w));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_incstate_step(const Grid &g, const T *q_in, const T *Df, const T *vt, const T *grad, T *q_out,
                                double cs, int last, T *b, double w, hipStream_t s) {
    hipLaunchKernelGGL(k_incstate_step<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, q_in, Df, vt, grad, q_out,
                       T(cs), last, b, T(w));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_incstate_init(const Grid &g, const T *vt, const T *grad, T *q, double cs, hipStream_t s) {
    hipLaunchKernelGGL(k_incstate_init<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g.N(), vt, grad, q, T(cs));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_deform_step(const Grid &g, const T *u_in, const T *Df, T *u_out, hipStream_t s) {
    const double pi2 = 6.283185307179586476925286766559;
    hipLaunchKernelGGL(k_deform_step<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, u_in, Df, u_out,
                       T(pi2 / g.n1), T(pi2 / g.n2), T(pi2 / g.n3));
    return hipGetLastError();
}

#define REGK_INST(T)                                                                                                 \
    template hipError_t launch_interp<T>(const Grid &, const T *, const T *, T *, hipStream_t);                      \
    template hipError_t launch_backtrace<T>(const Grid &, const T *, double, T *, hipStream_t);                      \
    template hipError_t launch_adjoint_step<T>(const Grid &, const T *, const T *, const T *, const T *, const T *,  \
                                               T *, T *, double, double, hipStream_t);                               \
    template hipError_t launch_adjoint_init<T>(const Grid &, const T *, const T *, const T *, T *, T *, double,      \
                                               hipStream_t);                                                         \
    template hipError_t launch_incstate_step<T>(const Grid &, const T *, const T *, const T *, const T *, T *,       \
                                                double, int, T *, double, hipStream_t);                              \
    template hipError_t launch_incstate_init<T>(const Grid &, const T *, const T *, T *, double, hipStream_t);       \
    template hipError_t launch_deform_step<T>(const Grid &, const T *, const T *, T *, hipStream_t);

REGK_INST(float)
REGK_INST(double)

}  // namespace regk
