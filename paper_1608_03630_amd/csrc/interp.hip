// Semi-Lagrangian transport kernels for gfx950: periodic tricubic Lagrange
// interpolation at departure points (sections III-B2 and III-C2 of the
// paper), the RK2 characteristic backtrace (eq. (6)) and the fused time-step
// kernels of the state, adjoint, incremental-state and incremental-adjoint
// solves (eq. (7)) and of the deformation map (eq. (1)).
//
// Every output point is computed by exactly one thread, which evaluates its
// 4x4x4 stencil separably (16 rows of 4 along x3, then 4 planes along x2,
// then x1): a race-free gather. Two forms:
// * the LDS-tiled kernels (the hot path): a workgroup stages the union of
//   its tile's stencils (a box known from the plan's floor bounds) in LDS
//   and reads every stencil value from there (see "LDS-staged tiles");
// * the direct gather (k_interp and friends, for displacements whose box
//   would not fit): each stencil row that does not wrap is one 16-byte
//   vector load (two for double), rows that wrap take four scalar loads.
// Blocks are remapped so that each XCD (8 per MI355X, one L2 each) receives
// a contiguous slab of the grid, which keeps the stencil halos of
// neighbouring blocks in the same L2.
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

// m mod n in [0, n); displacements are mostly within one period, so the
// division runs only for the rare far point
__device__ __forceinline__ int wrap_idx(int m, int n) {
    if (m < 0) m += n;
    else if (m >= n) m -= n;
    if ((unsigned)m >= (unsigned)n) {
        m %= n;
        if (m < 0) m += n;
    }
    return m;
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

// The stencil of one departure point: wrapped element offsets along x1 and
// x2, the first x3 index b3 of the rows (wrapped), the row length n3, and the
// per-axis weights.
template <typename T>
struct Stencil {
    int o1[4], o2[4];
    int b3, n3;
    T w1[4], w2[4], w3[4];
};

// first stencil index (m - 1 wrapped into [0, n)) and the weights of one axis
template <typename T>
__device__ __forceinline__ int axis_base(int i, T d, int n, T w[4]) {
    const T fl = flo(d);
    const T t = d - fl;  // exact
    // clamp before the conversion (NaN maps to the lower bound); the modulo
    // then keeps every stencil index inside [0, n)
    const T flc = fmin(fmax(fl, T(-1e9)), T(1e9));
    lagrange4(t, w);
    return wrap_idx(i + (int)flc - 1, n);  // |i + flc| < 2^31
}

__device__ __forceinline__ void axis_offsets(int base, int n, int stride, int o[4]) {
    int x = base;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        o[a] = x * stride;
        x = (x + 1 == n) ? 0 : x + 1;
    }
}

template <typename T>
__device__ __forceinline__ void make_stencil(const Grid &g, int i1, int i2, int i3, T d1, T d2, T d3,
                                             Stencil<T> &st) {
    axis_offsets(axis_base(i1, d1, g.n1, st.w1), g.n1, g.n2 * g.n3, st.o1);
    axis_offsets(axis_base(i2, d2, g.n2, st.w2), g.n2, g.n3, st.o2);
    st.b3 = axis_base(i3, d3, g.n3, st.w3);
    st.n3 = g.n3;
}

// 4 consecutive values of a row that does not wrap, as 16-byte loads at
// element (not vector) alignment
typedef float f4_unaligned __attribute__((ext_vector_type(4), aligned(4)));
typedef double d2_unaligned __attribute__((ext_vector_type(2), aligned(8)));


template <typename T> struct Row;
template <> struct Row<float> {
    f4_unaligned v;
    __device__ __forceinline__ void load(const float *p) { v = *reinterpret_cast<const f4_unaligned *>(p); }
    __device__ __forceinline__ float dot(const float w[4]) const { return w[0] * v.x + w[1] * v.y + w[2] * v.z + w[3] * v.w; }
};
template <> struct Row<double> {
    d2_unaligned a, b;
    __device__ __forceinline__ void load(const double *p) {
        a = *reinterpret_cast<const d2_unaligned *>(p);
        b = *reinterpret_cast<const d2_unaligned *>(p + 2);
    }
    __device__ __forceinline__ double dot(const double w[4]) const {
        return w[0] * a.x + w[1] * a.y + w[2] * b.x + w[3] * b.y;
    }
};

template <typename T>
__device__ __forceinline__ T apply(const T *__restrict__ f, const Stencil<T> &st) {
    T acc = T(0);
    if (st.b3 + 3 < st.n3) {
        // all 16 row loads are issued before the first use, so a wavefront
        // keeps 16 requests in flight instead of one
        Row<T> r[16];
#pragma unroll
        for (int a = 0; a < 4; a++)
#pragma unroll
            for (int b = 0; b < 4; b++) r[a * 4 + b].load(f + st.o1[a] + st.o2[b] + st.b3);
#pragma unroll
        for (int a = 0; a < 4; a++) {
            T pa = T(0);
#pragma unroll
            for (int b = 0; b < 4; b++) pa += st.w2[b] * r[a * 4 + b].dot(st.w3);
            acc += st.w1[a] * pa;
        }
    } else {
        int o3[4];
        axis_offsets(st.b3, st.n3, 1, o3);
#pragma unroll
        for (int a = 0; a < 4; a++) {
            T pa = T(0);
#pragma unroll
            for (int b = 0; b < 4; b++) {
                const T *row = f + st.o1[a] + st.o2[b];
                pa += st.w2[b] * (st.w3[0] * row[o3[0]] + st.w3[1] * row[o3[1]] + st.w3[2] * row[o3[2]] +
                                  st.w3[3] * row[o3[3]]);
            }
            acc += st.w1[a] * pa;
        }
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
// nu_new = nu0 + dt/2 (f0 + f*). The source is linear in nu, so the step is
// nu_new = nu(X) * gam(x) with gam = 1 + dt/2 (c(X) + c) + dt^2/2 c(X) c,
// formed once per plan (k_gamma); gam = null when div v = 0.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_step(Grid g, const T *__restrict__ lam_in,
                                                           const T *__restrict__ Da, const T *__restrict__ gam,
                                                           T *__restrict__ lam_out) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N(), p = pi.p;
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, Da[p], Da[N + p], Da[2 * N + p], st);
    T lam = apply(lam_in, st);
    if (gam) lam *= gam[p];
    lam_out[p] = lam;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_gamma(long N, const T *__restrict__ c, const T *__restrict__ cX,
                                                    T *__restrict__ gam, T dt) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    const T a = cX[p], b = c[p];
    gam[p] = T(1) + T(0.5) * dt * (a + b) + T(0.5) * dt * dt * a * b;
}

// b = sum_n w_n lam^n grad rho^n over the stored levels (trapezoid weights
// dt/2 at both ends, dt inside); pointwise in x, so one streaming pass
template <typename T>
__global__ __launch_bounds__(kThreads) void k_b_assemble(long N, int nt, const T *__restrict__ lam,
                                                         const T *__restrict__ grad, T *__restrict__ b) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    const T dt = T(1) / T(nt);
    T b1 = T(0), b2 = T(0), b3 = T(0);
    for (int k = 0; k <= nt; k++) {
        const T w = (k == 0 || k == nt) ? T(0.5) * dt : dt;
        const T s = w * __builtin_nontemporal_load(lam + (long)k * N + p);
        const T *gk = grad + (long)k * 3 * N;
        b1 += s * __builtin_nontemporal_load(gk + p);
        b2 += s * __builtin_nontemporal_load(gk + N + p);
        b3 += s * __builtin_nontemporal_load(gk + 2 * N + p);
    }
    b[p] = b1;
    b[N + p] = b2;
    b[2 * N + p] = b3;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_adjoint_init(long N, const T *__restrict__ rhoR,
                                                           const T *__restrict__ rho1, T *__restrict__ lam) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    lam[p] = rhoR[p] - rho1[p];
}

// q_out = q_in(X) + cs * (vt . grad rho^{n+1}); the last step writes
// lam~(1) = -(that), the start of the incremental adjoint.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_incstate_step(Grid g, const T *__restrict__ q_in,
                                                            const T *__restrict__ Df, const T *__restrict__ vt,
                                                            const T *__restrict__ grad, T *__restrict__ q_out, T cs,
                                                            int last) {
    PointIdx pi;
    if (!point_of(g, pi)) return;
    const long N = g.N(), p = pi.p;
    Stencil<T> st;
    make_stencil(g, pi.i1, pi.i2, pi.i3, Df[p], Df[N + p], Df[2 * N + p], st);
    const T s = vt[p] * grad[p] + vt[N + p] * grad[N + p] + vt[2 * N + p] * grad[2 * N + p];
    const T q = apply(q_in, st) + cs * s;
    q_out[p] = last ? -q : q;
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_incstate_init(long N, const T *__restrict__ vt,
                                                            const T *__restrict__ grad, T *__restrict__ q, T cs) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    if (p >= N) return;
    q[p] = cs * (__builtin_nontemporal_load(vt + p) * __builtin_nontemporal_load(grad + p) +
                 __builtin_nontemporal_load(vt + N + p) * __builtin_nontemporal_load(grad + N + p) +
                 __builtin_nontemporal_load(vt + 2 * N + p) * __builtin_nontemporal_load(grad + 2 * N + p));
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


// ---------------------------------------------------------- LDS-staged tiles
//
// A workgroup owns a kTile1 x kTile2 x kTile3 tile of output points. The
// union of their stencils is the box [tile origin + lo, + B) per axis, known
// from the floor bounds of D over the whole field (computed once per plan).
// The box is staged in LDS with coalesced row loads (wrapping periodically),
// then each point reads its 64 values from LDS at local indices that need no
// modulo; local indices are clamped to the box so that even a NaN
// displacement cannot address outside it.

constexpr int kTileLines = kTile1 * kTile2;       // x3 lines per tile
// Workgroup of the LDS-tiled gathers: kTileThreads threads share one tile's
// box, each owning kLinesPerWave x3 lines (points). A 4 x 8 x 64 tile with a
// padded box of 8 x 12 x 96 floats (36 KiB) lets four workgroups (32
// wavefronts, under 48 VGPRs each) share a CU.
constexpr int kTileThreads = 512;
constexpr int kWaves = kTileThreads / 64;
constexpr int kLinesPerWave = kTileLines / kWaves;

struct TileIdx {
    int t1, t2, t3;  // tile coordinates
};

__device__ __forceinline__ TileIdx tile_of(const Grid &g) {
    const int nt3 = (g.n3 + kTile3 - 1) / kTile3, nt2 = (g.n2 + kTile2 - 1) / kTile2;
    const unsigned b = (unsigned)xcd_block();
    TileIdx t;
    t.t3 = (int)(b % nt3);
    const unsigned r = b / nt3;
    t.t2 = (int)(r % nt2);
    t.t1 = (int)(r / nt2);
    return t;
}

// Global-memory view of a pointer. The tile bodies access fields through it:
// in the batched kernels the pointers are read from the work list, and with
// plain pointers the compiler, not knowing their address space, emitted flat
// loads and stores, whose completion the LDS wait counter also tracks (every
// LDS wait of the gather then waited for the streaming loads as well).
template <typename T> using gmem = __attribute__((address_space(1))) T;

// stage the box of field f for tile t into box[] (row-major [B1][B2][B3]).
// Rows are taken kStageRows at a time per wavefront and every value of the
// batch is requested before the first LDS store, so that each wavefront keeps
// up to kStageRows * 3 loads in flight (B3 <= 64 + 3 + 64 < 192).
constexpr int kStageRows = 4;

// Index of this thread's wavefront, in a scalar register: everything derived
// from it (rows to stage, row addresses) is then wave-uniform scalar work.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)); }

// Row (r1, r2) of a B1 x B2 row grid advanced by `step` rows (r2 fastest).
__device__ __forceinline__ void next_row(int &r1, int &r2, int step, int B2) {
    r2 += step;
    while (r2 >= B2) {
        r2 -= B2;
        r1++;
    }
}

template <typename T>
__device__ __forceinline__ void stage_box(const Grid &g, const TileGeom &tg, const TileIdx &t,
                                          const T *__restrict__ f, T *box) {
    const int o1 = t.t1 * kTile1 + tg.lo[0], o2 = t.t2 * kTile2 + tg.lo[1], o3 = t.t3 * kTile3 + tg.lo[2];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int B1 = tg.B[0], B2 = tg.B[1], B3 = tg.B[2];
    int gc[3];
#pragma unroll
    for (int h = 0; h < 3; h++) gc[h] = wrap_idx(o3 + lane + 64 * h, g.n3);
    int r1 = 0, r2 = 0;
    next_row(r1, r2, wave, B2);
    while (r1 < B1) {
        T vals[kStageRows][3];
        int dst[kStageRows];
        int q1 = r1, q2 = r2;
#pragma unroll
        for (int u = 0; u < kStageRows; u++) {
            dst[u] = -1;
            if (q1 < B1) {
                const int g1 = wrap_idx(o1 + q1, g.n1), g2 = wrap_idx(o2 + q2, g.n2);
                const gmem<T> *row = (const gmem<T> *)f + ((long)g1 * g.n2 + g2) * g.n3;
#pragma unroll
                for (int h = 0; h < 3; h++)
                    if (lane + 64 * h < B3) vals[u][h] = row[gc[h]];
                dst[u] = (q1 * B2 + q2) * B3;
            }
            next_row(q1, q2, kWaves, B2);
        }
#pragma unroll
        for (int u = 0; u < kStageRows; u++) {
            if (dst[u] >= 0) {
                T *d = box + dst[u];
#pragma unroll
                for (int h = 0; h < 3; h++)
                    if (lane + 64 * h < B3) d[lane + 64 * h] = vals[u][h];
            }
        }
        r1 = q1;
        r2 = q2;
    }
}

// local stencil start along one axis (clamped into the box) and the weights
template <typename T>
__device__ __forceinline__ int local_base(int il, T d, int lo, int B, T w[4]) {
    const T fl = flo(d);
    lagrange4(d - fl, w);
    const T flc = fmin(fmax(fl, T(-1e6)), T(1e6));
    const int l = il + (int)flc - 1 - lo;
    return min(max(l, 0), B - 4);
}

template <typename T>
__device__ __forceinline__ T apply_box(const T *box, const TileGeom &tg, int l1, int l2, int l3, const T w1[4],
                                       const T w2[4], const T w3[4]) {
    const int s2 = tg.B[2], s1 = tg.B[1] * tg.B[2];
    const T *base = box + l1 * s1 + l2 * s2 + l3;
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < 4; a++) {
        T pa = T(0);
#pragma unroll
        for (int b = 0; b < 4; b++) {
            const T *row = base + a * s1 + b * s2;
            pa += w2[b] * (w3[0] * row[0] + w3[1] * row[1] + w3[2] * row[2] + w3[3] * row[3]);
        }
        acc += w1[a] * pa;
    }
    return acc;
}

enum TileMode { TM_INTERP = 0, TM_ADJOINT = 1, TM_INCSTATE = 2 };

struct TileArgs {
    const void *gam, *grad, *vt;  // mode inputs (may be null)
    void *out;                    // output field
    double cs;
    int last;
};

// One body for the three gather-based time steps of one tile; the mode picks
// the epilogue (see k_interp, k_adjoint_step, k_incstate_step for the
// formulas). Each thread owns kLinesPerWave points (one per x3 line it
// visits); their displacements are loaded before the box is staged so that
// those HBM reads overlap the staging, and each point's epilogue operands are
// requested before its 64 LDS reads. Ragged tiles are masked point by point;
// every thread reaches the barrier.
template <typename T, int MODE>
__device__ __forceinline__ void generic_tile(const Grid &g, const TileGeom &tg, const TileIdx &t,
                                             const T *__restrict__ f, const T *__restrict__ D, const TileArgs &args,
                                             T *box) {
    const long N = g.N();
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int i3 = t.t3 * kTile3 + lane;
    const bool col_ok = i3 < g.n3;
    T dd[kLinesPerWave][3];
    long pp[kLinesPerWave];
#pragma unroll
    for (int k = 0; k < kLinesPerWave; k++) {
        const int line = wave + kWaves * k;
        const int a1 = line / kTile2, a2 = line - a1 * kTile2;
        const int i1 = t.t1 * kTile1 + a1, i2 = t.t2 * kTile2 + a2;
        const bool ok = col_ok && i1 < g.n1 && i2 < g.n2;
        const long p = ok ? ((long)i1 * g.n2 + i2) * g.n3 + i3 : -1;
        pp[k] = p;
        const gmem<T> *Dg = (const gmem<T> *)D;
        dd[k][0] = ok ? Dg[p] : T(0);
        dd[k][1] = ok ? Dg[N + p] : T(0);
        dd[k][2] = ok ? Dg[2 * N + p] : T(0);
    }
    stage_box(g, tg, t, f, box);
    __syncthreads();
    const gmem<T> *__restrict__ gam = (const gmem<T> *)args.gam;
    const gmem<T> *__restrict__ grad = (const gmem<T> *)args.grad;
    const gmem<T> *__restrict__ vt = (const gmem<T> *)args.vt;
    gmem<T> *__restrict__ out = (gmem<T> *)args.out;
#pragma unroll
    for (int k = 0; k < kLinesPerWave; k++) {
        const long p = pp[k];
        if (p < 0) continue;
        const int line = wave + kWaves * k;
        const int a1 = line / kTile2, a2 = line - a1 * kTile2;
        T e0 = T(1), sv = T(0);
        if (MODE == TM_ADJOINT) {
            if (gam) e0 = gam[p];
        } else if (MODE == TM_INCSTATE) {
            sv = vt[p] * grad[p] + vt[N + p] * grad[N + p] + vt[2 * N + p] * grad[2 * N + p];
        }
        T w1[4], w2[4], w3[4];
        const int l1 = local_base(a1, dd[k][0], tg.lo[0], tg.B[0], w1);
        const int l2 = local_base(a2, dd[k][1], tg.lo[1], tg.B[1], w2);
        const int l3 = local_base(lane, dd[k][2], tg.lo[2], tg.B[2], w3);
        T v = apply_box(box, tg, l1, l2, l3, w1, w2, w3);
        if (MODE == TM_INTERP) {
            out[p] = v;
        } else if (MODE == TM_ADJOINT) {
            out[p] = v * e0;
        } else {  // TM_INCSTATE
            v = v + T(args.cs) * sv;
            out[p] = args.last ? -v : v;
        }
    }
}

template <typename T, int MODE>
__global__ __launch_bounds__(kTileThreads) void k_tiled(Grid g, TileGeom tg, const T *__restrict__ f,
                                                    const T *__restrict__ D, TileArgs args) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    generic_tile<T, MODE>(g, tg, tile_of(g), f, D, args, reinterpret_cast<T *>(smem_raw));
}

// The same three time steps with compile-time box strides: the box is stored
// at the canonical extents kTile_j + 3 + S (any floor span <= S fits), so the
// 64 LDS reads of a stencil are immediate offsets from one address, all index
// arithmetic is 32-bit, and the per-thread point loop is fully unrolled with
// no per-point branches (interior tiles only; the launcher sends ragged tiles
// to k_tiled through the same grid via the `interior` test below).
constexpr int kCanonMaxSpan = 4;  // largest canonical box: (7+S)(11+S)(67+S) floats, padded, <= 64 KB

// Row pitch C3. LDS has 32 four-byte banks; lanes of a half-wavefront read
// consecutive x3 positions, and where the floor of D1 or D2 changes between
// them, some read the next row. With a pitch of 0 mod 32 those lanes keep
// distinct banks; with kTile3 + 3 + S (4 + S mod 32) they collide with the
// lanes of the first row, and with 16 mod 32 only lanes 16 apart can. The
// pitch is the multiple of 32, else of 16, else the natural one, whichever
// first reaches the most workgroups per CU (160 KiB of LDS, at most four
// 512-thread workgroups): 96 for span 1, 80 for spans 2 and 4.
// The tile is T1 x T2 x kTile3 (4 x 8 x 64 by default; the batched kernels
// also take the other shapes of kBatchTiles): 64 T2 threads, one x2 row per
// wavefront, T1 points (x1 rows) per thread. The workgroups per CU are capped
// by the 32 wavefronts a CU holds.
constexpr int kLdsPerCu = 160 * 1024;
template <int S, int T1 = kTile1, int T2 = kTile2> struct Canon {
    static constexpr int C1 = T1 + 3 + S, C2 = T2 + 3 + S, W = kTile3 + 3 + S;
    static constexpr int P32 = (W + 31) / 32 * 32, P16 = (W + 15) / 16 * 16;
    static constexpr int kMaxWg = 32 / T2;
    static constexpr int wg(int pitch) {
        const int bytes = C1 * C2 * pitch * 4;
        return bytes > 65536 ? 0 : (kLdsPerCu / bytes < kMaxWg ? kLdsPerCu / bytes : kMaxWg);
    }
    static constexpr int best = wg(W) > wg(P16) ? wg(W) : wg(P16);
    static constexpr int C3 = wg(P32) >= best ? P32 : wg(P16) >= best ? P16 : W;
    static constexpr int elems = C1 * C2 * C3;
    static constexpr bool fits = elems * 4 <= 65536;
};

template <typename T, int S, int T1 = kTile1, int T2 = kTile2>
__device__ __forceinline__ void stage_box_canon(const Grid &g, const TileGeom &tg, const TileIdx &t,
                                                const T *__restrict__ f, T *box) {
    using K = Canon<S, T1, T2>;
    constexpr int kW = T2;  // wavefronts of the workgroup
    const int o1 = t.t1 * T1 + tg.lo[0], o2 = t.t2 * T2 + tg.lo[1], o3 = t.t3 * kTile3 + tg.lo[2];
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const int B1 = tg.B[0], B2 = tg.B[1], B3 = tg.B[2];
    const int gc0 = wrap_idx(o3 + lane, g.n3), gc1 = wrap_idx(o3 + lane + 64, g.n3);
    const bool h1 = lane + 64 < B3;
    int r1 = 0, r2 = 0;
    next_row(r1, r2, wave, B2);
    while (r1 < B1) {
        T v0[kStageRows], v1[kStageRows];
        int dst[kStageRows];
        int q1 = r1, q2 = r2;
#pragma unroll
        for (int u = 0; u < kStageRows; u++) {
            dst[u] = -1;
            if (q1 < B1) {
                const int g1 = wrap_idx(o1 + q1, g.n1), g2 = wrap_idx(o2 + q2, g.n2);
                const gmem<T> *row = (const gmem<T> *)f + (unsigned)((g1 * g.n2 + g2) * g.n3);
                v0[u] = row[gc0];
                if (h1) v1[u] = row[gc1];
                dst[u] = (q1 * K::C2 + q2) * K::C3;
            }
            next_row(q1, q2, kW, B2);
        }
#pragma unroll
        for (int u = 0; u < kStageRows; u++) {
            if (dst[u] >= 0) {
                box[dst[u] + lane] = v0[u];
                if (h1) box[dst[u] + lane + 64] = v1[u];
            }
        }
        r1 = q1;
        r2 = q2;
    }
}

// The cubic Lagrange basis of lagrange4 times 6 (10 operations instead of
// 14); a stencil sum with three such factors is 216 times the interpolant.
template <typename T>
__device__ __forceinline__ void lagrange4_x6(T t, T w[4]) {
    const T tm1 = t - T(1), tm2 = t - T(2), tp1 = t + T(1);
    const T a = t * tm1;              // t (t - 1)
    const T c = (t * T(3) + T(3)) * tm2;  // 3 (t + 1) (t - 2)
    w[0] = -(a * tm2);
    w[1] = c * tm1;
    w[2] = -(c * t);
    w[3] = a * tp1;
}

// Local stencil start along one axis and the (scaled) weights. The floor is
// clamped in floating point to [flo_min, flo_min + B - 4], the floors whose
// stencil lies inside the box, so the index needs no integer clamp; a NaN
// displacement maps to flo_min (the clamp takes the non-NaN operand).
template <typename T>
__device__ __forceinline__ int canon_base(T d, T flo_min, T flo_max, int shift, T w[4]) {
    const T fl = flo(d);
    lagrange4_x6(d - fl, w);
    return (int)fmin(fmax(fl, flo_min), flo_max) + shift;
}

// Element at a 32-bit byte offset from a uniform base: the load or store
// then takes the scalar-base + 32-bit vector-offset address form (the
// canonical kernels run on single-precision grids of at most 2^30 points, so
// every field offset fits). Non-temporal for the per-point streams.
template <typename T>
__device__ __forceinline__ T ld_nt(const gmem<T> *base, unsigned byte_off) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const gmem<T> *>(reinterpret_cast<const gmem<char> *>(base) + byte_off));
}
template <typename T>
__device__ __forceinline__ void st_at(gmem<T> *base, unsigned byte_off, T v) {
    *reinterpret_cast<gmem<T> *>(reinterpret_cast<gmem<char> *>(base) + byte_off) = v;
}

// An integer the compiler must treat as unknown: the per-plane LDS offsets go
// through it so that each plane's 16 reads use immediate offsets from one
// register, instead of the compiler re-deriving a base per pair of reads from
// one folded offset (ds_read2 offsets reach only 255 elements).
__device__ __forceinline__ unsigned opaque(unsigned x) {
    asm("" : "+v"(x));
    return x;
}

// The work of one tile t of one grid (shared by the single-grid and the
// batched persistent kernels; `box` is the workgroup's LDS). The thread's
// displacements and Heun factors are requested before the box is staged, so
// that their HBM latency overlaps the staging; the six streams of vt . grad
// rho of the incremental-state step are read in the point loop instead (in
// the staging phase they lengthened it by 3%).
template <typename T, int MODE, int S, int T1 = kTile1, int T2 = kTile2>
__device__ __forceinline__ void canon_tile(const Grid &g, const TileGeom &tg, const TileIdx &t,
                                           const T *__restrict__ f, const T *__restrict__ D, const TileArgs &args,
                                           T *box) {
    using K = Canon<S, T1, T2>;
    static_assert(sizeof(T) == 4, "canonical tiles are single precision");
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const unsigned N = (unsigned)g.N();
    const gmem<T> *__restrict__ D1 = (const gmem<T> *)D;
    const gmem<T> *__restrict__ D2 = D1 + N;
    const gmem<T> *__restrict__ D3 = D1 + 2 * (size_t)N;
    const int i3 = t.t3 * kTile3 + lane;
    const unsigned line_bytes = (unsigned)g.n3 * sizeof(T);
    const unsigned b0 = (unsigned)(((t.t1 * T1) * g.n2 + t.t2 * T2) * g.n3 + i3) * sizeof(T);
    const gmem<T> *__restrict__ gam = (const gmem<T> *)args.gam;
    const gmem<T> *__restrict__ gr1 = (const gmem<T> *)args.grad;
    const gmem<T> *__restrict__ gr2 = gr1 + N;
    const gmem<T> *__restrict__ gr3 = gr1 + 2 * (size_t)N;
    const gmem<T> *__restrict__ vt1 = (const gmem<T> *)args.vt;
    const gmem<T> *__restrict__ vt2 = vt1 + N;
    const gmem<T> *__restrict__ vt3 = vt1 + 2 * (size_t)N;
    // thread's points: x1 row k = 0..T1-1 and x2 row `wave` of the tile, at
    // x3 position `lane`
    const int a2 = wave;
    T d[T1][3], e[T1];
#pragma unroll
    for (int k = 0; k < T1; k++) {
        const int a1 = k;
        const unsigned o = b0 + (unsigned)(a1 * g.n2 + a2) * line_bytes;
        d[k][0] = ld_nt(D1, o);
        d[k][1] = ld_nt(D2, o);
        d[k][2] = ld_nt(D3, o);
        if (MODE == TM_ADJOINT) {
            e[k] = gam ? ld_nt(gam, o) : T(1);
        }
    }
    stage_box_canon<T, S, T1, T2>(g, tg, t, f, box);
    __syncthreads();
    gmem<T> *__restrict__ out = (gmem<T> *)args.out;
    const T cs = T(args.cs);
    const bool last = args.last != 0;
    constexpr unsigned kPlane = K::C2 * K::C3;
    const T f3min = T(tg.lo[2] + 1 - lane), f3max = T(tg.lo[2] + tg.B[2] - 3 - lane);
#pragma unroll
    for (int k = 0; k < T1; k++) {
        const int a1 = k;
        const unsigned o = b0 + (unsigned)(a1 * g.n2 + a2) * line_bytes;
        // local start l = i_local + floor - 1 - lo, kept in [0, B - 4]
        T w1[4], w2[4], w3[4];
        const int l1 = canon_base(d[k][0], T(tg.lo[0] + 1 - a1), T(tg.lo[0] + tg.B[0] - 3 - a1), a1 - 1 - tg.lo[0], w1);
        const int l2 = canon_base(d[k][1], T(tg.lo[1] + 1 - a2), T(tg.lo[1] + tg.B[1] - 3 - a2), a2 - 1 - tg.lo[1], w2);
        const int l3 = canon_base(d[k][2], f3min, f3max, lane - 1 - tg.lo[2], w3);
        // byte offset of the stencil's first value; rows 0-2 of a plane are
        // read from one base and row 3 (beyond the 255-element reach of a
        // paired read) from a second one
        const unsigned eb = (unsigned)((l1 * K::C2 + l2) * K::C3 + l3) * sizeof(T);
        const char *lds = reinterpret_cast<const char *>(box);
        T acc = T(0);
#pragma unroll
        for (int a = 0; a < 4; a++) {
            const T *r0 = reinterpret_cast<const T *>(lds + opaque(eb + a * kPlane * sizeof(T)));
            const T *r3 = reinterpret_cast<const T *>(lds + opaque(eb + (a * kPlane + 3 * K::C3) * sizeof(T)));
            T v[4][4];
#pragma unroll
            for (int b = 0; b < 3; b++)
#pragma unroll
                for (int c = 0; c < 4; c++) v[b][c] = r0[b * K::C3 + c];
#pragma unroll
            for (int c = 0; c < 4; c++) v[3][c] = r3[c];
            T pa = T(0);
#pragma unroll
            for (int b = 0; b < 4; b++)
                pa += w2[b] * (w3[0] * v[b][0] + w3[1] * v[b][1] + w3[2] * v[b][2] + w3[3] * v[b][3]);
            acc += w1[a] * pa;
        }
        if (MODE == TM_INCSTATE)
            e[k] = ld_nt(vt1, o) * ld_nt(gr1, o) + ld_nt(vt2, o) * ld_nt(gr2, o) + ld_nt(vt3, o) * ld_nt(gr3, o);
        acc *= T(1.0 / 216.0);  // the three scaled weight factors
        if (MODE == TM_INTERP) {
            st_at(out, o, acc);
        } else if (MODE == TM_ADJOINT) {
            st_at(out, o, acc * e[k]);
        } else {
            const T v = acc + cs * e[k];
            st_at(out, o, last ? -v : v);
        }
    }
}

template <typename T, int MODE, int S>
__global__ __launch_bounds__(kTileThreads) void k_tiled_canon(Grid g, TileGeom tg, const T *__restrict__ f,
                                                          const T *__restrict__ D, TileArgs args) {
    __shared__ T box[Canon<S>::elems];
    canon_tile<T, MODE, S>(g, tg, tile_of(g), f, D, args, box);
}

// ------------------------------------------------ RK2 backtrace through LDS
//
// The departure points of eq. (6) need v at the predicted points x + D*,
// D* = c v(x) / h: three gathers with one stencil per point. A workgroup owns
// a canonical tile; from its points' predictors it reduces its own floor
// bounds (so one fast region does not widen every tile's box), then stages
// the three components of v one after another in that box and reads each
// point's stencil from LDS. A tile whose predictor spans more floors than the
// box holds, or is not finite, gathers straight from global memory. The
// result is D = c (v(x) + v(x + D*)) / (2 h).

// the stencil sum of v at one point's predicted position, from a staged
// canonical box (scaled weights, so the sum is divided by 216 at the end)
template <int S>
__device__ __forceinline__ float bt_point(const float *box, const TileGeom &tg, int a1, int a2, int lane, float d1,
                                          float d2, float d3) {
    using K = Canon<S>;
    constexpr unsigned kPlane = K::C2 * K::C3;
    float w1[4], w2[4], w3[4];
    const int l1 = canon_base(d1, float(tg.lo[0] + 1 - a1), float(tg.lo[0] + tg.B[0] - 3 - a1), a1 - 1 - tg.lo[0], w1);
    const int l2 = canon_base(d2, float(tg.lo[1] + 1 - a2), float(tg.lo[1] + tg.B[1] - 3 - a2), a2 - 1 - tg.lo[1], w2);
    const int l3 = canon_base(d3, float(tg.lo[2] + 1 - lane), float(tg.lo[2] + tg.B[2] - 3 - lane),
                              lane - 1 - tg.lo[2], w3);
    const unsigned eb = (unsigned)((l1 * K::C2 + l2) * K::C3 + l3) * sizeof(float);
    const char *lds = reinterpret_cast<const char *>(box);
    float acc = 0.f;
#pragma unroll
    for (int a = 0; a < 4; a++) {
        const float *r0 = reinterpret_cast<const float *>(lds + opaque(eb + a * kPlane * sizeof(float)));
        const float *r3 = reinterpret_cast<const float *>(lds + opaque(eb + (a * kPlane + 3 * K::C3) * sizeof(float)));
        float pa = 0.f;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            const float *r = r0 + b * K::C3;
            pa += w2[b] * (w3[0] * r[0] + w3[1] * r[1] + w3[2] * r[2] + w3[3] * r[3]);
        }
        pa += w2[3] * (w3[0] * r3[0] + w3[1] * r3[1] + w3[2] * r3[2] + w3[3] * r3[3]);
        acc += w1[a] * pa;
    }
    return acc * (1.f / 216.f);
}

// the three components through a box of span S, each written as soon as it
// is gathered
template <int S>
__device__ __forceinline__ void bt_tile_canon(const Grid &g, const TileGeom &tg, const TileIdx &t,
                                              const float *__restrict__ v, const float (&u)[kTile1][3], const float c,
                                              const float ih[3], float *box, float *__restrict__ D, unsigned b0,
                                              unsigned line_bytes) {
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const unsigned N = (unsigned)g.N();
    const float hc = 0.5f * c;
#pragma unroll
    for (int j = 0; j < 3; j++) {
        if (j) __syncthreads();  // the previous component's reads are done
        stage_box_canon<float, S>(g, tg, t, v + (size_t)j * N, box);
        __syncthreads();
        gmem<float> *__restrict__ out = (gmem<float> *)D + (size_t)j * N;
#pragma unroll
        for (int k = 0; k < kTile1; k++) {
            // the predictor again for each component, through an opaque copy:
            // otherwise the compiler keeps all points' weights alive across
            // the three stagings (120 registers instead of under 80)
            float d1 = c * u[k][0] * ih[0], d2 = c * u[k][1] * ih[1], d3 = c * u[k][2] * ih[2];
            asm("" : "+v"(d1), "+v"(d2), "+v"(d3));
            const float w = bt_point<S>(box, tg, k, wave, lane, d1, d2, d3);
            st_at(out, b0 + (unsigned)(k * g.n2 + wave) * line_bytes, hc * (u[k][j] + w) * ih[j]);
        }
    }
}

// Launched with eight wavefronts per SIMD requested, so that four workgroups
// share a CU as their LDS allows: the compiler then fits the kernel in 64
// registers with a few spilled (at its natural 80 registers only three fit,
// and a 256^3 backtrace took 413 instead of 380 us).
__global__ __launch_bounds__(kTileThreads, 8) void k_backtrace_canon(Grid g, const float *__restrict__ v, float c,
                                                                  float ih1, float ih2, float ih3,
                                                                  float *__restrict__ D) {
    constexpr int kElems = Canon<1>::elems > Canon<2>::elems ? Canon<1>::elems : Canon<2>::elems;
    __shared__ float box[kElems];
    __shared__ float red[kWaves][6];
    const TileIdx t = tile_of(g);
    const int wave = wave_id(), lane = threadIdx.x & 63;
    const unsigned N = (unsigned)g.N();
    const unsigned line_bytes = (unsigned)g.n3 * sizeof(float);
    const int i3 = t.t3 * kTile3 + lane;
    const unsigned b0 = (unsigned)(((t.t1 * kTile1) * g.n2 + t.t2 * kTile2) * g.n3 + i3) * sizeof(float);
    const float ih[3] = {ih1, ih2, ih3};
    // the thread's points (x1 rows k, x2 row `wave`, x3 position `lane`):
    // ordinary loads, so that the lines stay in L2 for the staging below
    const gmem<float> *V = (const gmem<float> *)v;
    float u[kTile1][3];
    float mn[3], mx[3];
#pragma unroll
    for (int k = 0; k < kTile1; k++) {
        const unsigned o = b0 + (unsigned)(k * g.n2 + wave) * line_bytes;
#pragma unroll
        for (int j = 0; j < 3; j++) {
            u[k][j] = *reinterpret_cast<const gmem<float> *>(reinterpret_cast<const gmem<char> *>(V + (size_t)j * N) + o);
            // floor of the predictor, clamped (NaN and infinities become
            // +-1e6, which no box holds)
            const float fl = floorf(c * u[k][j] * ih[j]);
            const float f = fl == fl ? fminf(fmaxf(fl, -1e6f), 1e6f) : 1e6f;
            mn[j] = k ? fminf(mn[j], f) : f;
            mx[j] = k ? fmaxf(mx[j], f) : f;
        }
    }
    // the tile's floor bounds: wavefront, then workgroup
#pragma unroll
    for (int j = 0; j < 3; j++) {
        for (int off = 32; off > 0; off >>= 1) {
            mn[j] = fminf(mn[j], __shfl_xor(mn[j], off, 64));
            mx[j] = fmaxf(mx[j], __shfl_xor(mx[j], off, 64));
        }
    }
    if (lane == 0) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            red[wave][2 * j] = mn[j];
            red[wave][2 * j + 1] = mx[j];
        }
    }
    __syncthreads();
    float lo[3], hi[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        lo[j] = red[0][2 * j];
        hi[j] = red[0][2 * j + 1];
#pragma unroll
        for (int w = 1; w < kWaves; w++) {
            lo[j] = fminf(lo[j], red[w][2 * j]);
            hi[j] = fmaxf(hi[j], red[w][2 * j + 1]);
        }
    }
    const float span = fmaxf(fmaxf(hi[0] - lo[0], hi[1] - lo[1]), hi[2] - lo[2]);
    if (span <= 2.f) {
        TileGeom tg;
        const int tile[3] = {kTile1, kTile2, kTile3};
#pragma unroll
        for (int j = 0; j < 3; j++) {
            tg.lo[j] = (int)lo[j] - 1;
            tg.B[j] = tile[j] + (int)(hi[j] - lo[j]) + 3;
        }
        if (span <= 1.f)
            bt_tile_canon<1>(g, tg, t, v, u, c, ih, box, D, b0, line_bytes);
        else
            bt_tile_canon<2>(g, tg, t, v, u, c, ih, box, D, b0, line_bytes);
        return;
    }
    // rare: one point, one component and one x1 plane at a time (operands
    // reloaded or recomputed, not indexed from unrolled arrays), so that the
    // loads of this path do not set the register budget of the kernel
    const float hc = 0.5f * c;
    const int i1_0 = t.t1 * kTile1, i2 = t.t2 * kTile2 + wave;
#pragma unroll 1
    for (int k = 0; k < kTile1; k++) {
        const unsigned o = b0 + (unsigned)(k * g.n2 + wave) * line_bytes;
        const unsigned p = o / sizeof(float);
        const float x1 = v[p], x2 = v[N + p], x3 = v[2 * (size_t)N + p];
        float w1[4], w2[4], w3[4];
        const int s1 = axis_base(i1_0 + k, c * x1 * ih1, g.n1, w1);
        int o2[4], o3[4];
        axis_offsets(axis_base(i2, c * x2 * ih2, g.n2, w2), g.n2, g.n3, o2);
        axis_offsets(axis_base(i3, c * x3 * ih3, g.n3, w3), g.n3, 1, o3);
#pragma unroll 1
        for (int j = 0; j < 3; j++) {
            // 32-bit byte offsets from the component's uniform base (grids
            // of the canonical kernels hold at most 2^30 points)
            const gmem<char> *f = reinterpret_cast<const gmem<char> *>((const gmem<float> *)v + (size_t)j * N);
            float w = 0.f;
            int r1 = s1;
#pragma unroll 1
            for (int a = 0; a < 4; a++) {
                const float wa = a == 0 ? w1[0] : a == 1 ? w1[1] : a == 2 ? w1[2] : w1[3];
                float pa = 0.f;
#pragma unroll
                for (int b = 0; b < 4; b++) {
                    const unsigned row = (unsigned)(r1 * g.n2 * g.n3 + o2[b]) * sizeof(float);
                    float x[4];
#pragma unroll
                    for (int q = 0; q < 4; q++)
                        x[q] = *reinterpret_cast<const gmem<float> *>(f + row + (unsigned)o3[q] * sizeof(float));
                    pa += w2[b] * (w3[0] * x[0] + w3[1] * x[1] + w3[2] * x[2] + w3[3] * x[3]);
                }
                w += wa * pa;
                r1 = r1 + 1 == g.n1 ? 0 : r1 + 1;
            }
            const float xj = j == 0 ? x1 : j == 1 ? x2 : x3, ihj = j == 0 ? ih1 : j == 1 ? ih2 : ih3;
            st_at((gmem<float> *)D + (size_t)j * N, o, hc * (xj + w) * ihj);
        }
    }
}

// Batched persistent variants: gridDim.x workgroups walk a work list of
// (pair, tile) items over all pairs of a batch (pairs sorted by tile0). With
// `chunked` the items are dealt to the XCDs in contiguous chunks, so that each
// XCD's L2 sees neighbouring tiles of one grid; otherwise round-robin. The
// per-tile work is that of the single-grid kernels (same arithmetic, so a
// pair's result does not depend on the batch).
// Work items count tiles of the launch's shape T1 x T2 x kTile3; the pair
// table's tile0 counts RATIO times as many: the smallest batch tile
// (kUnit1 x kUnit2 x kTile3, of which a canonical launch tile holds
// (T1 / kUnit1) (T2 / kUnit2)), or for the generic kernel the default tile
// itself (RATIO 1, ragged grids). The pair's box extents are those of the
// default tile, adjusted to T1 and T2.
template <int T1, int T2, int RATIO, class F>
__device__ __forceinline__ void walk_items(const PairStep *__restrict__ pairs, int npairs, int total, int chunked,
                                           F &&work) {
    constexpr int ratio = RATIO;
    const int nb = gridDim.x;
    int first = 0, end = total, stride = nb, start = blockIdx.x;
    if (chunked) {
        const int x = blockIdx.x % kXcds;
        stride = nb / kXcds + (x < nb % kXcds ? 1 : 0);
        start = blockIdx.x / kXcds;
        const int chunk = (total + kXcds - 1) / kXcds;
        first = x * chunk;
        end = min(total, first + chunk);
    }
    // A workgroup's items increase, so the pair that holds them (the last
    // with tile0 <= item) only moves forward: one binary search for the first
    // item, then a linear advance, and the pair record is read again only
    // when the pair changes.
    int item = first + start;
    if (item >= end) return;
    int lo = 0, hi = npairs - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pairs[mid].tile0 / ratio <= item) lo = mid;
        else hi = mid - 1;
    }
    auto load = [&](int i) {
        PairStep p = pairs[i];
        p.tg.B[0] += T1 - kTile1;
        p.tg.B[1] += T2 - kTile2;
        return p;
    };
    PairStep ps = load(lo);
    int next0 = lo + 1 < npairs ? pairs[lo + 1].tile0 / ratio : total;
    for (; item < end; item += stride) {
        if (item >= next0) {
            while (lo + 1 < npairs && pairs[lo + 1].tile0 / ratio <= item) lo++;
            ps = load(lo);
            next0 = lo + 1 < npairs ? pairs[lo + 1].tile0 / ratio : total;
        }
        const Grid g = ps.g;
        const int b = item - ps.tile0 / ratio;
        const int nt3 = (g.n3 + kTile3 - 1) / kTile3, nt2 = (g.n2 + T2 - 1) / T2;
        TileIdx t;
        t.t3 = b % nt3;
        t.t2 = (b / nt3) % nt2;
        t.t1 = b / (nt3 * nt2);
        TileArgs a;
        a.gam = ps.gam;
        a.grad = ps.grad;
        a.vt = ps.vt;
        a.out = ps.out;
        a.cs = ps.cs;
        a.last = ps.last;
        work(g, ps.tg, t, ps.f, ps.D, a);
        __syncthreads();  // the next item restages the box
    }
}

template <typename T, int MODE, int S, int T1, int T2>
__global__ __launch_bounds__(64 * T2) void k_batched_canon(const PairStep *__restrict__ pairs, int npairs, int total,
                                                           int chunked) {
    __shared__ T box[Canon<S, T1, T2>::elems];
    walk_items<T1, T2, (T1 / kUnit1) * (T2 / kUnit2)>(pairs, npairs, total, chunked,
                       [&](const Grid &g, const TileGeom &tg, const TileIdx &t, const void *f, const void *D,
                           const TileArgs &a) {
                           canon_tile<T, MODE, S, T1, T2>(g, tg, t, static_cast<const T *>(f),
                                                          static_cast<const T *>(D), a, box);
                       });
}

// The generic body for every pair (dynamic LDS sized for the largest box).
template <typename T, int MODE>
__global__ __launch_bounds__(kTileThreads) void k_batched_generic(const PairStep *__restrict__ pairs, int npairs,
                                                              int total, int chunked) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *box = reinterpret_cast<T *>(smem_raw);
    walk_items<kTile1, kTile2, 1>(pairs, npairs, total, chunked,
                               [&](const Grid &g, const TileGeom &tg, const TileIdx &t, const void *f, const void *D,
                                   const TileArgs &a) {
                                   generic_tile<T, MODE>(g, tg, t, static_cast<const T *>(f),
                                                         static_cast<const T *>(D), a, box);
                               });
}

// Floor bounds of D, one partial per block. Wide blocks with four loads per
// stream in flight: the partial buffer allows only RED_BLOCKS / 6 blocks, and
// with 256 threads those kept too few loads in flight to stream D at HBM
// rate. Floors are exact in T, so min and max are taken in T; NaN entries
// are skipped (the gathers clamp their floors into the box).
constexpr int kBoundThreads = 1024;

template <typename T>
__global__ __launch_bounds__(kBoundThreads) void k_floor_bounds(Grid g, const T *__restrict__ D,
                                                                double *__restrict__ partials) {
    const long N = g.N();
    const long stride = (long)gridDim.x * kBoundThreads;
    T mn[3], mx[3];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        mn[j] = T(INFINITY);
        mx[j] = T(-INFINITY);
    }
    long i = (long)blockIdx.x * kBoundThreads + threadIdx.x;
    for (; i + 3 * stride < N; i += 4 * stride) {
        T x[3][4];
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int u = 0; u < 4; u++) x[j][u] = D[j * N + i + u * stride];
#pragma unroll
        for (int j = 0; j < 3; j++)
#pragma unroll
            for (int u = 0; u < 4; u++) {
                const T fl = flo(x[j][u]);
                mn[j] = fmin(mn[j], fl);
                mx[j] = fmax(mx[j], fl);
            }
    }
    for (; i < N; i += stride) {
#pragma unroll
        for (int j = 0; j < 3; j++) {
            const T fl = flo(D[j * N + i]);
            mn[j] = fmin(mn[j], fl);
            mx[j] = fmax(mx[j], fl);
        }
    }
    __shared__ T sm[6][kBoundThreads / 64];
#pragma unroll
    for (int j = 0; j < 3; j++) {
        for (int off = 32; off > 0; off >>= 1) {
            mn[j] = fmin(mn[j], __shfl_down(mn[j], off, 64));
            mx[j] = fmax(mx[j], __shfl_down(mx[j], off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            sm[2 * j][threadIdx.x >> 6] = mn[j];
            sm[2 * j + 1][threadIdx.x >> 6] = mx[j];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const bool is_min = (threadIdx.x & 1) == 0;
        T v = sm[threadIdx.x][0];
        for (int w = 1; w < kBoundThreads / 64; w++) v = is_min ? fmin(v, sm[threadIdx.x][w]) : fmax(v, sm[threadIdx.x][w]);
        partials[6 * blockIdx.x + threadIdx.x] = (double)v;
    }
}

__global__ void k_finalize_bounds(const double *__restrict__ partials, int nblocks, double *__restrict__ out6) {
    if (threadIdx.x < 6) {
        const bool is_min = (threadIdx.x & 1) == 0;
        double v = partials[threadIdx.x];
        for (int b = 1; b < nblocks; b++) {
            const double x = partials[6 * b + threadIdx.x];
            v = is_min ? fmin(v, x) : fmax(v, x);
        }
        out6[threadIdx.x] = v;
    }
}

inline unsigned ntiles(const Grid &g) {
    return (unsigned)(((g.n1 + kTile1 - 1) / kTile1) * ((g.n2 + kTile2 - 1) / kTile2) *
                      ((g.n3 + kTile3 - 1) / kTile3));
}

// largest floor span of a box
inline int box_span(const TileGeom &tg) {
    return max(max(tg.B[0] - kTile1, tg.B[1] - kTile2), tg.B[2] - kTile3) - 3;
}

template <typename T, int MODE>
hipError_t launch_tiled(const Grid &g, const TileGeom &tg, const T *f, const T *D, const TileArgs &a, hipStream_t s) {
    // canonical-stride kernels need whole tiles (every grid extent a multiple
    // of the tile) and a floor span the canonical box holds
    const bool whole = g.n1 % kTile1 == 0 && g.n2 % kTile2 == 0 && g.n3 % kTile3 == 0;
    const int span = box_span(tg);
    if constexpr (sizeof(T) == 4) {
        if (whole && span <= 1) {
            hipLaunchKernelGGL((k_tiled_canon<T, MODE, 1>), dim3(ntiles(g)), dim3(kTileThreads), 0, s, g, tg, f, D, a);
            return hipGetLastError();
        }
        if (whole && span <= 2) {
            hipLaunchKernelGGL((k_tiled_canon<T, MODE, 2>), dim3(ntiles(g)), dim3(kTileThreads), 0, s, g, tg, f, D, a);
            return hipGetLastError();
        }
        if (whole && span <= kCanonMaxSpan) {
            hipLaunchKernelGGL((k_tiled_canon<T, MODE, kCanonMaxSpan>), dim3(ntiles(g)), dim3(kTileThreads), 0, s, g, tg,
                               f, D, a);
            return hipGetLastError();
        }
    }
    const size_t lds = sizeof(T) * (size_t)tg.B[0] * tg.B[1] * tg.B[2];
    hipLaunchKernelGGL((k_tiled<T, MODE>), dim3(ntiles(g)), dim3(kTileThreads), lds, s, g, tg, f, D, a);
    return hipGetLastError();
}

inline unsigned nblocks(long N) { return (unsigned)((N + kThreads - 1) / kThreads); }

}  // namespace

bool canonical(const Grid &g, const TileGeom &tg, size_t esz) {
    return esz == 4 && g.n1 % kTile1 == 0 && g.n2 % kTile2 == 0 && g.n3 % kTile3 == 0 &&
           box_span(tg) <= kCanonMaxSpan;
}

int batch_span(const TileGeom &tg) { return box_span(tg); }

int tiles_of(const Grid &g) { return (int)ntiles(g); }

int unit_tiles_of(const Grid &g) {
    return ((g.n1 + kUnit1 - 1) / kUnit1) * ((g.n2 + kUnit2 - 1) / kUnit2) * ((g.n3 + kTile3 - 1) / kTile3);
}

namespace {

// the canonical batched kernel of one tile shape, mode and span
template <int M, int S, int T1, int T2>
hipError_t launch_canon_shape(const PairStep *pairs, int npairs, int total, int nb, int chunked, hipStream_t s) {
    if constexpr (Canon<S, T1, T2>::fits) {
        hipLaunchKernelGGL((k_batched_canon<float, M, S, T1, T2>), dim3(nb), dim3(64 * T2), 0, s, pairs, npairs, total,
                           chunked);
        return hipGetLastError();
    } else {
        return hipErrorInvalidValue;
    }
}

template <int M, int S>
hipError_t launch_canon_tile(int t1, int t2, const PairStep *pairs, int npairs, int total, int nb, int chunked,
                             hipStream_t s) {
    if (t1 == 4 && t2 == 8) return launch_canon_shape<M, S, 4, 8>(pairs, npairs, total, nb, chunked, s);
    if (t1 == 2 && t2 == 8) return launch_canon_shape<M, S, 2, 8>(pairs, npairs, total, nb, chunked, s);
    if (t1 == 8 && t2 == 8) return launch_canon_shape<M, S, 8, 8>(pairs, npairs, total, nb, chunked, s);
    if (t1 == 4 && t2 == 4) return launch_canon_shape<M, S, 4, 4>(pairs, npairs, total, nb, chunked, s);
    if (t1 == 8 && t2 == 4) return launch_canon_shape<M, S, 8, 4>(pairs, npairs, total, nb, chunked, s);
    return hipErrorInvalidValue;
}

template <int M>
hipError_t launch_canon_mode(int variant, int t1, int t2, const PairStep *pairs, int npairs, int total, int nb,
                             int chunked, hipStream_t s) {
    if (variant == 1) return launch_canon_tile<M, 1>(t1, t2, pairs, npairs, total, nb, chunked, s);
    if (variant == 2) return launch_canon_tile<M, 2>(t1, t2, pairs, npairs, total, nb, chunked, s);
    return launch_canon_tile<M, kCanonMaxSpan>(t1, t2, pairs, npairs, total, nb, chunked, s);
}

}  // namespace

namespace {
template <int S>
bool canon_fits(int t1, int t2) {
    if (t1 == 4 && t2 == 8) return Canon<S, 4, 8>::fits;
    if (t1 == 2 && t2 == 8) return Canon<S, 2, 8>::fits;
    if (t1 == 8 && t2 == 8) return Canon<S, 8, 8>::fits;
    if (t1 == 4 && t2 == 4) return Canon<S, 4, 4>::fits;
    if (t1 == 8 && t2 == 4) return Canon<S, 8, 4>::fits;
    return false;
}
}  // namespace

bool batch_tile_ok(int variant, int t1, int t2) {
    if (variant == 0) return t1 == kTile1 && t2 == kTile2;
    if (variant == 1) return canon_fits<1>(t1, t2);
    if (variant == 2) return canon_fits<2>(t1, t2);
    return canon_fits<kCanonMaxSpan>(t1, t2);
}

template <typename T>
hipError_t launch_batched_step(int mode, int variant, size_t lds, const PairStep *pairs_dev, int npairs, int total,
                               int nblocks_grid, int chunked, int t1, int t2, hipStream_t s) {
    // chunked dealing needs a workgroup on every XCD
    if (npairs < 1 || total < 1 || nblocks_grid < kXcds) return hipErrorInvalidValue;
    const bool canon_variant = variant == 1 || variant == 2 || variant == kCanonMaxSpan;
    if (!canon_variant && variant != 0) return hipErrorInvalidValue;
    if (variant == 0 && (lds == 0 || lds > 65536 || t1 != kTile1 || t2 != kTile2)) return hipErrorInvalidValue;
    if (variant != 0 && sizeof(T) != 4) return hipErrorInvalidValue;
    if (variant == 0) {
        const dim3 grid(nblocks_grid), block(kTileThreads);
        if (mode == TM_INTERP)
            hipLaunchKernelGGL((k_batched_generic<T, TM_INTERP>), grid, block, lds, s, pairs_dev, npairs, total, chunked);
        else if (mode == TM_ADJOINT)
            hipLaunchKernelGGL((k_batched_generic<T, TM_ADJOINT>), grid, block, lds, s, pairs_dev, npairs, total, chunked);
        else
            hipLaunchKernelGGL((k_batched_generic<T, TM_INCSTATE>), grid, block, lds, s, pairs_dev, npairs, total, chunked);
        return hipGetLastError();
    }
    if (mode == TM_INTERP) return launch_canon_mode<TM_INTERP>(variant, t1, t2, pairs_dev, npairs, total, nblocks_grid, chunked, s);
    if (mode == TM_ADJOINT) return launch_canon_mode<TM_ADJOINT>(variant, t1, t2, pairs_dev, npairs, total, nblocks_grid, chunked, s);
    return launch_canon_mode<TM_INCSTATE>(variant, t1, t2, pairs_dev, npairs, total, nblocks_grid, chunked, s);
}

template hipError_t launch_batched_step<float>(int, int, size_t, const PairStep *, int, int, int, int, int, int,
                                               hipStream_t);
template hipError_t launch_batched_step<double>(int, int, size_t, const PairStep *, int, int, int, int, int, int,
                                                hipStream_t);

namespace {

}  // namespace

// ---------------------------------------------------------------- launchers

bool tile_geom(const double fmin[3], const double fmax[3], size_t elem, TileGeom *tg) {
    const int T[3] = {kTile1, kTile2, kTile3};
    size_t vol = elem;
    for (int j = 0; j < 3; j++) {
        const double span = fmax[j] - fmin[j];
        // the staging loop covers rows of up to 192 values: B3 = 67 + span
        if (!(span >= 0) || span > 64 || !(fabs(fmin[j]) < 1e6)) return false;
        tg->lo[j] = (int)fmin[j] - 1;
        tg->B[j] = T[j] + (int)span + 3;
        vol *= (size_t)tg->B[j];
    }
    return vol <= 65536;
}

template <typename T>
hipError_t launch_floor_bounds(const Grid &g, const T *D, double *partials, int nb, hipStream_t s) {
    hipLaunchKernelGGL(k_floor_bounds<T>, dim3(nb), dim3(kBoundThreads), 0, s, g, D, partials);
    return hipGetLastError();
}

hipError_t launch_finalize_bounds(const double *partials, int nb, double *out6, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize_bounds, dim3(1), dim3(64), 0, s, partials, nb, out6);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_interp(const Grid &g, const T *f, const T *D, T *out, hipStream_t s, const TileGeom *tg) {
    if (tg) {
        TileArgs a{};
        a.out = out;
        return launch_tiled<T, TM_INTERP>(g, *tg, f, D, a, s);
    }
    hipLaunchKernelGGL(k_interp<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, f, D, out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_backtrace(const Grid &g, const T *v, double sign_dt, T *D, hipStream_t s) {
    const double pi2 = 6.283185307179586476925286766559;
    if constexpr (sizeof(T) == 4) {
        // whole canonical tiles: the LDS form
        if (g.n1 % kTile1 == 0 && g.n2 % kTile2 == 0 && g.n3 % kTile3 == 0) {
            hipLaunchKernelGGL(k_backtrace_canon, dim3(ntiles(g)), dim3(kTileThreads), 0, s, g, v, T(-sign_dt),
                               T(g.n1 / pi2), T(g.n2 / pi2), T(g.n3 / pi2), D);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_backtrace<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, v, T(-sign_dt),
                       T(g.n1 / pi2), T(g.n2 / pi2), T(g.n3 / pi2), D);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_step(const Grid &g, const T *lam_in, const T *Da, const T *gam, T *lam_out, hipStream_t s,
                               const TileGeom *tg) {
    if (tg) {
        TileArgs a{};
        a.gam = gam;
        a.out = lam_out;
        return launch_tiled<T, TM_ADJOINT>(g, *tg, lam_in, Da, a, s);
    }
    hipLaunchKernelGGL(k_adjoint_step<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, lam_in, Da, gam, lam_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gamma(long N, const T *c, const T *cX, T *gam, double dt, hipStream_t s) {
    hipLaunchKernelGGL(k_gamma<T>, dim3(nblocks(N)), dim3(kThreads), 0, s, N, c, cX, gam, T(dt));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_b_assemble(long N, int nt, const T *lam, const T *grad, T *b, hipStream_t s) {
    hipLaunchKernelGGL(k_b_assemble<T>, dim3(nblocks(N)), dim3(kThreads), 0, s, N, nt, lam, grad, b);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_init(long N, const T *rhoR, const T *rho1, T *lam, hipStream_t s) {
    hipLaunchKernelGGL(k_adjoint_init<T>, dim3(nblocks(N)), dim3(kThreads), 0, s, N, rhoR, rho1, lam);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_incstate_step(const Grid &g, const T *q_in, const T *Df, const T *vt, const T *grad, T *q_out,
                                double cs, int last, hipStream_t s, const TileGeom *tg) {
    if (tg) {
        TileArgs a{};
        a.vt = vt;
        a.grad = grad;
        a.out = q_out;
        a.cs = cs;
        a.last = last;
        return launch_tiled<T, TM_INCSTATE>(g, *tg, q_in, Df, a, s);
    }
    hipLaunchKernelGGL(k_incstate_step<T>, dim3(nblocks(g.N())), dim3(kThreads), 0, s, g, q_in, Df, vt, grad, q_out,
                       T(cs), last);
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
    template hipError_t launch_interp<T>(const Grid &, const T *, const T *, T *, hipStream_t, const TileGeom *);    \
    template hipError_t launch_floor_bounds<T>(const Grid &, const T *, double *, int, hipStream_t);                 \
    template hipError_t launch_backtrace<T>(const Grid &, const T *, double, T *, hipStream_t);                      \
    template hipError_t launch_adjoint_step<T>(const Grid &, const T *, const T *, const T *, T *, hipStream_t,      \
                                               const TileGeom *);                                                    \
    template hipError_t launch_gamma<T>(long, const T *, const T *, T *, double, hipStream_t);                       \
    template hipError_t launch_b_assemble<T>(long, int, const T *, const T *, T *, hipStream_t);                     \
    template hipError_t launch_adjoint_init<T>(long, const T *, const T *, T *, hipStream_t);                        \
    template hipError_t launch_incstate_step<T>(const Grid &, const T *, const T *, const T *, const T *, T *,       \
                                                double, int, hipStream_t, const TileGeom *);                         \
    template hipError_t launch_incstate_init<T>(const Grid &, const T *, const T *, T *, double, hipStream_t);       \
    template hipError_t launch_deform_step<T>(const Grid &, const T *, const T *, T *, hipStream_t);

REGK_INST(float)
REGK_INST(double)

}  // namespace regk
