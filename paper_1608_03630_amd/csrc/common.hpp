// Internal declarations shared by the HIP translation units of libreg.
// Grid geometry, complex helpers and the host-side launchers that the C ABI
// layer (capi.hip) drives. Nothing here is part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace regk {

// A regular periodic grid [n1][n2][n3], x3 fastest.
struct Grid {
    int n1, n2, n3;
    __host__ __device__ long N() const { return (long)n1 * n2 * n3; }
    __host__ __device__ int n3h() const { return n3 / 2 + 1; }
    __host__ __device__ long Nh() const { return (long)n1 * n2 * n3h(); }
};

template <typename T> struct cplx_of;
template <> struct cplx_of<float> { using type = float2; };
template <> struct cplx_of<double> { using type = double2; };
template <typename T> using cplx_t = typename cplx_of<T>::type;

// Radix plan of one line length: radices 8, then 4, 2, 3 and 5 (Stockham order).
struct FftPlan {
    int n;
    int npass;
    int radix[12];
};

bool make_plan(int n, FftPlan *p);

// ------------------------------------------------------------------ interp.hip
// Output tile of the LDS-staged gathers and the bounding box of its stencils.
constexpr int kTile1 = 4, kTile2 = 8, kTile3 = 64;
struct TileGeom {
    int lo[3];  // floor(min D_j) - 1: box origin relative to the tile origin
    int B[3];   // box extent per axis: tile + (floor(max D_j) - floor(min D_j)) + 3
};
// A box of this geometry fits the LDS budget of the tiled kernels.
bool tile_geom(const double fmin[3], const double fmax[3], size_t elem, TileGeom *tg);
// Per-block min and max of floor(D_j) for the three components
// (partials[6*b + 2j] = min, [6*b + 2j + 1] = max); nblocks blocks.
template <typename T>
hipError_t launch_floor_bounds(const Grid &g, const T *D, double *partials, int nblocks, hipStream_t s);
hipError_t launch_finalize_bounds(const double *partials, int nblocks, double *out6, hipStream_t s);

// One pair's operands of a batched transport step (single precision): the
// gathered field f, displacements D, mode operands, output, and the first
// work item of its tiles in the batch's work list.
struct PairStep {
    Grid g;
    TileGeom tg;
    const void *f, *D, *gam, *grad, *vt;
    void *out;
    double cs;
    int last;
    int tile0;
    int canon;  // the pair's gathers can take the canonical kernels
};
enum { STEP_INTERP = 0, STEP_ADJOINT = 1, STEP_INCSTATE = 2 };
// Grids whose gathers the canonical-stride LDS kernels take (single
// precision, whole 4x8x64 tiles, floor span of the box <= 4); any grid with a
// tile geometry can go through the generic kernels.
bool canonical(const Grid &g, const TileGeom &tg, size_t esz);
int batch_span(const TileGeom &tg);
int tiles_of(const Grid &g);
// Tile shapes T1 x T2 x 64 of the batched canonical kernels (64 T2 threads,
// T1 points per thread); the pair table counts tiles of the smallest,
// kUnit1 x kUnit2 x 64 (unit_tiles_of), so that every shape's tile index
// follows from it. A shape serves a launch when every pair's n1 and n2 are
// multiples of it and the box of the variant fits 64 KB (batch_tile_ok).
constexpr int kUnit1 = 2, kUnit2 = 4;
constexpr int kBatchTileCount = 5;
constexpr int kBatchTiles[kBatchTileCount][2] = {{4, 8}, {2, 8}, {8, 8}, {4, 4}, {8, 4}};
int unit_tiles_of(const Grid &g);
bool batch_tile_ok(int variant, int t1, int t2);
// One persistent launch of nblocks workgroups (>= 8) over all pairs' tiles
// (pairs_dev sorted by tile0, total = sum of the pairs' tiles). variant 0:
// generic tile kernel with `lds` bytes of dynamic LDS (the largest box of the
// pairs); variant 1, 2, 4: canonical box of that span (float only, every pair
// canonical with span <= variant). Tile shape t1 x t2 x 64 (the generic
// variant takes the default 4 x 8 only); total counts tiles of that shape.
template <typename T>
hipError_t launch_batched_step(int mode, int variant, size_t lds, const PairStep *pairs_dev, int npairs, int total,
                               int nblocks, int chunked, int t1, int t2, hipStream_t s);

// Every launcher enqueues on `s` and returns the hipError_t of the launch. A
// non-null TileGeom selects the LDS-staged gather for displacements D whose
// floor bounds it was built from; null selects the direct gather.
template <typename T>
hipError_t launch_interp(const Grid &g, const T *f, const T *D, T *out, hipStream_t s,
                         const TileGeom *tg = nullptr);
template <typename T>
hipError_t launch_backtrace(const Grid &g, const T *v, double sign_dt, T *D, hipStream_t s);
// adjoint-type step: lam_out = lam_in(X) * gam (gam = null: pure interpolation)
template <typename T>
hipError_t launch_adjoint_step(const Grid &g, const T *lam_in, const T *Da, const T *gam, T *lam_out, hipStream_t s,
                               const TileGeom *tg = nullptr);
// gam = 1 + dt/2 (cX + c) + dt^2/2 cX c: the Heun factor of the adjoint source
template <typename T>
hipError_t launch_gamma(long N, const T *c, const T *cX, T *gam, double dt, hipStream_t s);
// b = sum_n w_n lam^n grad^n (trapezoid weights) from nt+1 stored levels
template <typename T>
hipError_t launch_b_assemble(long N, int nt, const T *lam, const T *grad, T *b, hipStream_t s);
// lam = rhoR - rho1
template <typename T>
hipError_t launch_adjoint_init(long N, const T *rhoR, const T *rho1, T *lam, hipStream_t s);
// incremental state: q_out = interp(q_in, Df) + cs * (vt . grad); with last,
// q_out = -(that) = lam~(1)
template <typename T>
hipError_t launch_incstate_step(const Grid &g, const T *q_in, const T *Df, const T *vt, const T *grad, T *q_out,
                                double cs, int last, hipStream_t s, const TileGeom *tg = nullptr);
template <typename T>
hipError_t launch_incstate_init(const Grid &g, const T *vt, const T *grad, T *q, double cs, hipStream_t s);
template <typename T>
hipError_t launch_deform_step(const Grid &g, const T *u_in, const T *Df, T *u_out, hipStream_t s);

// --------------------------------------------------------------------- fft.hip
struct SpecCtx {
    Grid g;
    FftPlan plan[3];
    const void *tw[2][3];  // per-axis twiddles exp(-2 pi i m / n_axis): [0] float2, [1] double2
    void *H;               // half-spectrum buffer of up to 6 complex components (sized for double)
};
// derivative along axis of ncomp fields u + k*in_stride into out + k*out_stride
// (accumulate: out += d_axis u)
template <typename T>
hipError_t spec_deriv(const SpecCtx &c, int axis, const T *u, long in_stride, T *out, long out_stride, int accumulate,
                      int ncomp, hipStream_t s);
// forward 3D real FFT of ncomp fields of type Tr, computed in T, into H
// components [h0, h0+ncomp)
template <typename Tr, typename T>
hipError_t spec_forward(const SpecCtx &c, const Tr *x, int ncomp, int h0, hipStream_t s);
// inverse 3D FFT (computed in T) of H components [0, ncomp) into real fields
// of type Tr (divides by N)
template <typename T, typename Tr>
hipError_t spec_inverse(const SpecCtx &c, Tr *out, int ncomp, hipStream_t s);

enum SymbolOp {
    SYM_BIHARM = 0,      // H_c *= a |k|^4
    SYM_INVBIHARM = 1,   // H_c *= 1/(a |k|^4), 1 at k = 0
    SYM_GAUSS = 2,       // H_c *= exp(-a^2 |k|^2 / 2)
    SYM_LERAY = 3,       // H_0..2 = P H_0..2
    SYM_PRECOND = 4,     // inverse biharmonic, then P if flag
    SYM_ASSEMBLE = 5     // H_c = a |k|^4 H_c + [P] H_{3+c}, c < 3
};
template <typename T>
hipError_t spec_symbol(const SpecCtx &c, int op, double a, int ncomp, int leray, hipStream_t s);
// H of dst (first ncomp components) = resampled H of src (Fourier truncation
// or zero padding, scaled by Nd/Ns)
template <typename T>
hipError_t spec_resample(const SpecCtx &src, const SpecCtx &dst, int ncomp, hipStream_t s);
// the same with explicit spectral buffers (the inverse overwrites Hin)
template <typename Tr, typename T>
hipError_t spec_forward_to(const SpecCtx &c, const Tr *x, int ncomp, void *Hout, hipStream_t s);
// src (nullptr: Hin) is read by the first pass, so that a spectrum held
// elsewhere is transformed without a copy into Hin
template <typename T, typename Tr>
hipError_t spec_inverse_from(const SpecCtx &c, void *Hin, Tr *out, int ncomp, hipStream_t s,
                             const void *src = nullptr);

// Spectral velocity vectors: [3][Nh] complex double (Nh = n1 n2 (n3/2+1)),
// the unnormalised forward transforms of real fields.
enum VecOp {
    VEC_ASSEMBLE = 0,  // out = a |k|^4 x + [P] y   (y: 3 complex-T components, e.g. a transformed field)
    VEC_PRECOND = 1,   // out = x / (a |k|^4) (x at k = 0), then [P]
    VEC_LERAY = 2      // out = P x
};
// H (3 complex-T components) = vhat
template <typename T>
hipError_t vec_load(const SpecCtx &c, const double *vhat, void *H, hipStream_t s);
// pointwise operator (out may alias x)
template <typename T>
hipError_t vec_symbol(const SpecCtx &c, int op, const double *x, const void *y, double a, int leray, double *out,
                      hipStream_t s);
// Fused Krylov passes (partials: one double per block of a grid-stride loop
// over the half spectrum, nblocks blocks). The PCG vectors s, r, p are stored
// as complex T ([3][Nh]: double with double fields, float with float
// fields); updates are computed in double and rounded when stored. The
// Hessian matvec of a direction p starts with the inverse transform of p
// read in place (spec_inverse_from with src = p); z = M r is never stored.
// s = 0, r = -g, p = M r; partials of <r, M r>
template <typename T>
hipError_t pcg_start(const SpecCtx &c, const double *g, double beta, int leray, void *s, void *r, void *p,
                     double *part_rz, int nblocks, hipStream_t st);
// with q = beta |k|^4 p + [P] y (y: the transformed b~ in H): s += a p,
// r -= a q; partials of <r, r> and <r, M r>
template <typename T>
hipError_t pcg_step(const SpecCtx &c, double a, const void *p, const void *y, double beta, int leray, void *s, void *r,
                    double *part_rr, double *part_rz, int nblocks, hipStream_t st);
// p = M r + b p
template <typename T>
hipError_t pcg_direction(const SpecCtx &c, const void *r, double b, double beta, int leray, void *p, hipStream_t st);
// partials of <p, beta |k|^4 p + [P] y> for a Krylov vector p
template <typename T>
hipError_t krylov_curvature(const SpecCtx &c, const void *p, const void *y, double beta, int leray, double *part,
                            int nblocks, hipStream_t st);
// partials of sum w(k3) Re(a conj b), a a velocity vector, b a Krylov vector
template <typename T>
hipError_t krylov_dot_partials(const SpecCtx &c, const double *a, const void *b, double *partials, int nblocks,
                               hipStream_t s);
// out = x + a y, x and out velocity vectors, y a Krylov vector
template <typename T>
hipError_t krylov_axpy(const SpecCtx &c, const double *x, double a, const void *y, double *out, hipStream_t s);
// out = a |k|^4 x + [P] y with partials of <x, out> (dot 1) or <out, out> (dot 2);
// out may be null (partials only)
template <typename T>
hipError_t vec_assemble_dot(const SpecCtx &c, const double *x, const void *y, double a, int leray, int dot, double *out,
                            double *part, int nblocks, hipStream_t st);
// partials of sum w(k3) Re(a conj b) (mode 0) or sum w(k3) |k|^4 |a|^2 (mode 1)
hipError_t vec_dot_partials(const SpecCtx &c, int mode, const double *a, const double *b, double *partials,
                            int nblocks, hipStream_t s);

// -------------------------------------------------------------------- blas.hip
constexpr int RED_BLOCKS = 1024;
constexpr int RED_THREADS = 256;
// partials[b] = sum over block b of a*b (mode 0), (a-b)^2 (mode 1), a*a (mode 2)
template <typename T>
hipError_t launch_dot_partials(const T *a, const T *b, long n, int mode, double *partials, hipStream_t s);
// out[slot] = scale * sum(partials[0..nparts)) in a fixed order
hipError_t launch_finalize(const double *partials, int nparts, double scale, double *out, hipStream_t s);
// det(I + grad u) per point from du[9][N] (du[a*3+b] = d_b u_a); per-block min and max
template <typename T>
hipError_t launch_det_partials(const T *du, long n, double *pmin, double *pmax, T *det_out, hipStream_t s);
hipError_t launch_finalize_minmax(const double *pmin, const double *pmax, int nparts, double *out2, hipStream_t s);
template <typename T>
hipError_t launch_fill(long n, double val, T *y, hipStream_t s);
template <typename T>
hipError_t launch_copy(long n, const T *x, T *y, hipStream_t s);
// y = (To) x, element by element
template <typename Ti, typename To>
hipError_t launch_convert(long n, const Ti *x, To *y, hipStream_t s);
// full Newton matvec: out_j = lam vt_j (3 components); q += cs (vt . g);
// out += s(X) dt/2 (1 + dt c) + dt/2 s_next (c null: 0); b_j += w lam g_j;
// y = a x
template <typename T>
hipError_t launch_scale_vec(long n, const T *lam, const T *vt, T *out, hipStream_t s);
template <typename T>
hipError_t launch_add_vdotgrad(long n, const T *vt, const T *g, T *q, double cs, hipStream_t s);
template <typename T>
hipError_t launch_newton_source(long n, const T *sX, const T *s_next, const T *c, double dt, T *out, hipStream_t s);
template <typename T>
hipError_t launch_b_axpy(long n, double w, const T *lam, const T *g, T *b, hipStream_t s);
template <typename T>
hipError_t launch_scale(long n, double a, const T *x, T *y, hipStream_t s);
// zero padding of an m[0] x m[1] x m[2] image into the centre of grid g
// (offset (n - m) / 2 per axis), and the crop of that block back out
template <typename T>
hipError_t launch_pad(const Grid &g, const int m[3], const T *img, T *out, hipStream_t s);
template <typename T>
hipError_t launch_crop(const Grid &g, const int m[3], const T *f, T *out, hipStream_t s);

}  // namespace regk
