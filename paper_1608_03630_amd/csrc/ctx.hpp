// Internal state of a registration context and the host-side building
// blocks shared by the operator entry points (capi.hip) and the
// Gauss-Newton-Krylov driver and its batched executor (solver.hip). Host code
// only orchestrates: every grid-sized operation runs in the kernels of
// interp.hip, fft.hip and blas.hip; the host reads back double-precision
// scalars (inner products, objective, norms) where the Newton-Krylov
// iteration branches on them.
//
// Precision: image-space fields (images, state and adjoint histories, grad
// rho, departure points, b) use the field type T of params.prec; the
// velocity-space vectors (v, g, the PCG vectors) are always double and the 3D
// spectral operators that act on them (lap^2, its inverse, P, the gradient
// and matvec assembly) run in double. The H2 regulariser multiplies the
// representation error of v by |k|^4 (up to (n sqrt(3)/2)^4, about 2.4e9 on
// a 256^3 grid), which single precision cannot absorb; the transport, whose
// data are smooth images, runs in T.
#pragma once
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/reg.h"
#include "common.hpp"

using regk::Grid;

namespace regc {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr size_t kAlign = 256;
constexpr int kSlots = 32;  // device result slots (doubles)

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

inline bool fft_friendly(int n) {
    if (n < 8 || n > 1024 || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

// Carves the workspace: every view is kAlign-aligned. With base == nullptr it
// only measures.
struct Layout {
    char *base;
    size_t off = 0;
    explicit Layout(char *b) : base(b) {}
    void *take(size_t bytes) {
        void *p = base ? base + off : nullptr;
        off += align_up(bytes);
        return p;
    }
};

// Times launches with event pairs on one stream; the pairs are resolved into
// per-kind totals after the stream has been synchronised.
struct Profiler {
    struct Rec {
        hipEvent_t a, b, pre;
        int kind;
    };
    hipStream_t stream = nullptr;
    bool on = false;
    int every = 1;                  // time one launch in `every` of each kind
    int64_t seen[REG_K_COUNT] = {0};  // launches of each kind since enabled
    std::vector<hipEvent_t> free_;
    std::vector<Rec> pending;
    double ms[REG_K_COUNT] = {0};
    int64_t n[REG_K_COUNT] = {0};

    void resolve() {
        for (auto &r : pending) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
                ms[r.kind] += t;
                n[r.kind] += 1;
            } else {
                (void)hipGetLastError();
            }
            free_.push_back(r.a);
            free_.push_back(r.b);
            if (r.pre) free_.push_back(r.pre);
        }
        pending.clear();
    }
    hipEvent_t take() {
        if (free_.empty()) {
            hipEvent_t e = nullptr;
            // timing only, read after a stream synchronisation: no
            // system-scope fence (which would write back and invalidate the
            // caches around every timed launch)
            if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
                (void)hipGetLastError();
                return nullptr;
            }
            return e;
        }
        hipEvent_t e = free_.back();
        free_.pop_back();
        return e;
    }
    void reset() {
        for (int k = 0; k < REG_K_COUNT; k++) {
            ms[k] = 0;
            n[k] = 0;
            seen[k] = 0;
        }
    }
    void release() {
        resolve();
        for (hipEvent_t e : free_) (void)hipEventDestroy(e);
        free_.clear();
    }
};

}  // namespace regc

#define DISPATCH(ctx, fn, ...) ((ctx)->P.prec ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

#define CTX_OK(ctx)                                   \
    do {                                              \
        if (!(ctx)) return REG_EINVAL;                \
        (ctx)->err.clear();                           \
    } while (0)

struct reg_ctx {
    reg_params P;
    hipStream_t stream = nullptr;
    int device = 0;
    Grid g{};
    regk::SpecCtx spec{};
    size_t esz = 4;
    long N = 0, Nh = 0;
    double beta = 0;

    // workspace views
    void *rhoT, *rhoR, *histA, *histB, *grho, *Df, *Da, *Dt, *c, *cX, *c2, *cX2, *lam[2], *bvec;
    long grho_levels = 0;  // levels of grad rho^n the workspace holds: nt + 1, or 1 (recomputed)
    void *lamh;        // adjoint levels lam^0..lam^nt
    void *lamg;        // full Newton: the adjoint levels of the last gradient (null otherwise)
    void *gam, *gam2;  // Heun factor of the adjoint source (cached plan, scratch plan)
    void *vf, *vtf;                                            // velocity copies in the field type
    // velocity space, spectral: [3][Nh] complex double (see vec_symbol)
    void *vhat, *ghat, *shat, *rhat, *zhat, *phat, *qhat, *vthat;
    void *u0, *u1, *du, *H;
    void *tw32[3], *tw64[3];
    double *dpart, *dpart2, *dres;
    double *hres = nullptr;  // pinned host mirror of dres

    regc::Profiler prof;  // event pairs around launches (reg_profile)

    // tile geometry of the LDS-staged gathers, per displacement buffer
    struct PlanGeom {
        const void *D = nullptr;
        bool tiled = false;
        regk::TileGeom tg{};
    };
    PlanGeom geoms[6];

    // grid continuation: the context of the grid coarsened by 2 per axis
    // (owned, its workspace follows this one's), and whether its images are
    // the restriction of the current ones
    reg_ctx *coarse = nullptr;
    bool coarse_images = false;

    bool have_images = false;
    bool have_state = false;  // plans, history, grad rho and div v at vhat
    double normTR2 = 0;       // <rho_T - rho_R, rho_T - rho_R>
    long interps = 0;
    int64_t fft3d = 0, fft_lines = 0;  // 3D transforms and line-FFT derivatives (one component/field each)
    double alg_bytes = 0;              // algorithmic HBM bytes of the kernels launched (see alg_fields)
    reg_log_fn log_fn = nullptr;       // progress log of the solves (reg_set_log)
    void *log_user = nullptr;
    int64_t epoch = 0;  // bumped whenever a plan (departure points, tile geometry) changes
    std::string err;
};

namespace regc {

inline reg_status fail(reg_ctx *ctx, reg_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

inline reg_status hipfail(reg_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, REG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                         \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hipfail((ctx), e_, #expr);  \
    } while (0)

// Runs one launcher; with profiling on, brackets every `every`-th launch of
// each kind with two events (an event pair costs a few microseconds of idle
// GPU between launches, so a long run samples). When sampling, a third event
// goes first: the first event after a kernel absorbs the wait for that
// kernel, and without it the sampled times ran 5% long.
template <class F>
hipError_t timed(Profiler &pr, int kind, F &&launch) {
    if (!pr.on || pr.seen[kind]++ % pr.every != 0) return launch();
    if (pr.pending.size() >= 8192) {
        hipError_t e = hipStreamSynchronize(pr.stream);
        if (e != hipSuccess) return e;
        pr.resolve();
    }
    hipEvent_t a = pr.take(), b = pr.take();
    hipEvent_t pre = pr.every > 1 ? pr.take() : nullptr;
    if (!a || !b || (pr.every > 1 && !pre)) {
        for (hipEvent_t x : {a, b, pre})
            if (x) pr.free_.push_back(x);
        return launch();
    }
    hipError_t e = hipSuccess;
    if (pre) {
        e = hipEventRecord(pre, pr.stream);
        if (e != hipSuccess) return e;
    }
    e = hipEventRecord(a, pr.stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, pr.stream);
    if (e != hipSuccess) return e;
    pr.pending.push_back({a, b, pre, kind});
    return hipSuccess;
}

#define KL(ctx, kind, expr) timed((ctx)->prof, (kind), [&]() { return (expr); })


#define STCHK(expr)                     \
    do {                                \
        reg_status s_ = (expr);         \
        if (s_ != REG_OK) return s_;    \
    } while (0)

inline reg_status check_params(const reg_params *p, std::string *why) {
    if (!p) {
        *why = "params is NULL";
        return REG_EINVAL;
    }
    for (int j = 0; j < 3; j++)
        if (!fft_friendly(p->n[j])) {
            *why = "grid size n[" + std::to_string(j) + "] = " + std::to_string(p->n[j]) +
                   " must be even, 2^a 3^b 5^c and in [8, 1024]";
            return REG_EINVAL;
        }
    if (p->nt < 1 || p->nt > 4096) {
        *why = "nt must be in [1, 4096]";
        return REG_EINVAL;
    }
    if (!(p->beta > 0) || !std::isfinite(p->beta)) {
        *why = "beta must be positive and finite";
        return REG_EINVAL;
    }
    if (p->prec != 0 && p->prec != 1) {
        *why = "prec must be 0 (float) or 1 (double)";
        return REG_EINVAL;
    }
    if (p->max_newton < 0 || p->max_pcg < 1 || p->max_ls < 0) {
        *why = "max_newton >= 0, max_pcg >= 1 and max_ls >= 0 are required";
        return REG_EINVAL;
    }
    if (!(p->gtol >= 0) || !(p->mismatch_tol >= 0)) {
        *why = "gtol and mismatch_tol must be >= 0";
        return REG_EINVAL;
    }
    if (!(p->gnorm_ref >= 0) || !std::isfinite(p->gnorm_ref)) {
        *why = "gnorm_ref must be >= 0 and finite";
        return REG_EINVAL;
    }
    if (!(p->gtol_level >= 0) || !std::isfinite(p->gtol_level)) {
        *why = "gtol_level must be >= 0 and finite";
        return REG_EINVAL;
    }
    if (p->det_check != 0 && p->det_check != 1) {
        *why = "det_check must be 0 or 1";
        return REG_EINVAL;
    }
    if (p->hessian != 0 && p->hessian != 1) {
        *why = "hessian must be 0 (Gauss-Newton) or 1 (full Newton)";
        return REG_EINVAL;
    }
    if (p->recompute_grad_rho != 0 && p->recompute_grad_rho != 1) {
        *why = "recompute_grad_rho must be 0 or 1";
        return REG_EINVAL;
    }
    if (p->recompute_grad_rho && p->hessian) {
        *why = "the full Newton Hessian (hessian = 1) needs grad rho of every level (recompute_grad_rho = 0)";
        return REG_EINVAL;
    }
    if (p->grid_levels < 0 || p->grid_levels > REG_MAXLEVELS) {
        *why = "grid_levels must be in [0, " + std::to_string(REG_MAXLEVELS) + "]";
        return REG_EINVAL;
    }
    for (int l = 1; l < p->grid_levels; l++)
        for (int j = 0; j < 3; j++)
            if ((p->n[j] % (1 << l)) != 0 || !fft_friendly(p->n[j] >> l)) {
                *why = "grid_levels = " + std::to_string(p->grid_levels) + " needs n[" + std::to_string(j) +
                       "] / " + std::to_string(1 << l) + " to be a valid grid size";
                return REG_EINVAL;
            }
    return REG_OK;
}

// grids of the continuation (1 = the context's own grid only)
inline int grid_count(const reg_params *p) { return p->grid_levels > 1 ? p->grid_levels : 1; }

// the settings of p on the grid coarsened by 2 per axis, one level fewer
inline reg_params coarse_params(const reg_params *p) {
    reg_params q = *p;
    for (int j = 0; j < 3; j++) q.n[j] = p->n[j] / 2;
    q.grid_levels = grid_count(p) - 1;
    return q;
}

// Lays out the workspace of a context (ctx == nullptr: size only).
inline size_t layout(const reg_params *p, char *base, reg_ctx *ctx) {
    const size_t E = p->prec ? 8 : 4;
    const long N = (long)p->n[0] * p->n[1] * p->n[2];
    const long Nh = (long)p->n[0] * p->n[1] * (p->n[2] / 2 + 1);
    const long nt1 = p->nt + 1;
    Layout L(base);
    reg_ctx tmp;
    reg_ctx *c = ctx ? ctx : &tmp;
    c->rhoT = L.take(E * N);
    c->rhoR = L.take(E * N);
    c->histA = L.take(E * N * nt1);
    c->histB = L.take(E * N * nt1);
    c->grho_levels = p->recompute_grad_rho ? 1 : nt1;
    c->grho = L.take(E * 3 * N * c->grho_levels);
    c->Df = L.take(E * 3 * N);
    c->Da = L.take(E * 3 * N);
    c->Dt = L.take(E * 3 * N);
    c->c = L.take(E * N);
    c->cX = L.take(E * N);
    c->c2 = L.take(E * N);
    c->cX2 = L.take(E * N);
    c->lam[0] = L.take(E * N);
    c->lam[1] = L.take(E * N);
    c->lamh = L.take(E * N * nt1);
    c->lamg = p->hessian ? L.take(E * N * nt1) : nullptr;
    c->gam = L.take(E * N);
    c->gam2 = L.take(E * N);
    c->bvec = L.take(E * 3 * N);
    c->vf = L.take(E * 3 * N);
    c->vtf = L.take(E * 3 * N);
    const size_t D8 = sizeof(double);
    const size_t SV = 2 * D8 * 3 * Nh;
    c->vhat = L.take(SV);
    c->ghat = L.take(SV);
    c->shat = L.take(SV);
    c->rhat = L.take(SV);
    c->zhat = L.take(SV);
    c->phat = L.take(SV);
    c->qhat = L.take(SV);
    c->vthat = L.take(SV);
    c->u0 = L.take(E * 3 * N);
    c->u1 = L.take(E * 3 * N);
    c->du = L.take(E * 9 * N);
    c->H = L.take(2 * D8 * 6 * Nh);
    for (int j = 0; j < 3; j++) {
        c->tw32[j] = L.take(2 * sizeof(float) * p->n[j]);
        c->tw64[j] = L.take(2 * D8 * p->n[j]);
    }
    c->dpart = (double *)L.take(sizeof(double) * regk::RED_BLOCKS);
    c->dpart2 = (double *)L.take(sizeof(double) * regk::RED_BLOCKS);
    c->dres = (double *)L.take(sizeof(double) * kSlots);
    return L.off;
}

// workspace of a context and of its coarse-grid chain
inline size_t total_size(const reg_params *p) {
    size_t b = align_up(layout(p, nullptr, nullptr));
    if (grid_count(p) > 1) {
        const reg_params q = coarse_params(p);
        b += total_size(&q);
    }
    return b;
}

inline bool is_device_ptr(const void *ptr) {
    if (!ptr) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, ptr) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged;
}

#define NEED_DEV(ctx, ptr)                                                                   \
    do {                                                                                     \
        if (!is_device_ptr(ptr)) return fail((ctx), REG_EINVAL, #ptr " is not a device pointer"); \
    } while (0)

// ------------------------------------------------------------ typed helpers

template <typename T> T *V(void *p) { return static_cast<T *>(p); }
template <typename T> const T *CV(const void *p) { return static_cast<const T *>(p); }

inline double h3(const reg_ctx *c) { return (kTwoPi / c->g.n1) * (kTwoPi / c->g.n2) * (kTwoPi / c->g.n3); }

inline const regk::TileGeom *geom_of(const reg_ctx *ctx, const void *D) {
    for (const auto &g : ctx->geoms)
        if (g.D == D) return g.tiled ? &g.tg : nullptr;
    return nullptr;
}

inline void set_geom(reg_ctx *ctx, const void *D, bool tiled, const regk::TileGeom &tg) {
    for (auto &g : ctx->geoms)
        if (g.D == D) {
            g.tiled = tiled;
            g.tg = tg;
            return;
        }
    for (auto &g : ctx->geoms)
        if (g.D == nullptr) {
            g.D = D;
            g.tiled = tiled;
            g.tg = tg;
            return;
        }
    ctx->geoms[0].D = D;  // table full: reuse a slot
    ctx->geoms[0].tiled = tiled;
    ctx->geoms[0].tg = tg;
}

// velocity (double) -> field type copy
template <typename T>
hipError_t to_field(reg_ctx *ctx, const void *src, void *dst, long n) {
    if (sizeof(T) == sizeof(double))
        return regk::launch_copy<double>(n, CV<double>(src), V<double>(dst), ctx->stream);
    return regk::launch_convert<double, float>(n, CV<double>(src), V<float>(dst), ctx->stream);
}

// Algorithmic HBM bytes: what each launched kernel must read and write at
// least (each operand once), summed per launch for reg_report.alg_bytes; a
// model from the operand sizes, not a counter reading. Fields count N
// elements, velocity-space vectors 3 Nh complex values, of the given type.
inline void alg_fields(reg_ctx *ctx, double fields, size_t esz) {
    ctx->alg_bytes += fields * (double)ctx->N * (double)esz;
}
inline void alg_fields(reg_ctx *ctx, double fields) { alg_fields(ctx, fields, ctx->esz); }
inline void alg_vecs(reg_ctx *ctx, double vectors, size_t esz) {
    ctx->alg_bytes += vectors * 6.0 * (double)ctx->Nh * (double)esz;
}
// ncomp 3D real transforms in a type of esz bytes: the x3 pass reads the
// real field and writes the half spectrum, each of the two strided passes
// reads and writes it in place
inline void alg_fft3d(reg_ctx *ctx, int ncomp, size_t esz) {
    ctx->alg_bytes += ncomp * ((double)ctx->N + 10.0 * (double)ctx->Nh) * (double)esz;
}

// reads kSlots doubles back (synchronises)
inline reg_status fetch(reg_ctx *ctx, int nslots) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * nslots, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!ctx->prof.pending.empty()) ctx->prof.resolve();
    return REG_OK;
}

// dres[slot] = scale * reduction
template <typename T>
reg_status reduce(reg_ctx *ctx, const void *a, const void *b, long n, int mode, double scale, int slot) {
    ctx->alg_bytes += (b ? 2.0 : 1.0) * (double)n * sizeof(T);
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_dot_partials<T>(CV<T>(a), CV<T>(b ? b : a), n, mode, ctx->dpart, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, scale, ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// Device result slots: 0 inner products, 1 mismatch numerator, 2 regulariser,
// 3 |g|^2, 4 a second inner product, 8..13 and 16..21 the floor bounds of two
// plans measured together.
constexpr int kSlotPlanA = 8, kSlotPlanB = 16;

// floor bounds of D over the grid into dres[slot..slot+5] (partials in `part`)
template <typename T>
reg_status bounds_enqueue(reg_ctx *ctx, const void *D, double *part, int slot) {
    alg_fields(ctx, 3);
    const int nb = regk::RED_BLOCKS / 6;
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_floor_bounds<T>(ctx->g, CV<T>(D), part, nb, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize_bounds(part, nb, ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// tile geometry of the gathers that use D, from bounds already in hres
inline void plan_finish(reg_ctx *ctx, const void *D, int slot) {
    double fmin[3], fmax[3];
    for (int j = 0; j < 3; j++) {
        fmin[j] = ctx->hres[slot + 2 * j];
        fmax[j] = ctx->hres[slot + 2 * j + 1];
    }
    regk::TileGeom tg{};
    const bool ok = regk::tile_geom(fmin, fmax, ctx->esz, &tg);
    set_geom(ctx, D, ok, tg);
    ctx->epoch++;
}

// departure points D of the field-type velocity vf (RK2 backtrace, sign +1
// forward in t, -1 for the adjoint) and their floor bounds
template <typename T>
reg_status plan_enqueue(reg_ctx *ctx, const void *vf, double sign, void *D, double *part, int slot) {
    HIPCHK(ctx, KL(ctx, REG_K_BACKTRACE, regk::launch_backtrace<T>(ctx->g, CV<T>(vf), sign / ctx->P.nt, V<T>(D), ctx->stream)));
    ctx->interps += 3;
    alg_fields(ctx, 6);  // v in, D out (the gathers' halos come from cache)
    return bounds_enqueue<T>(ctx, D, part, slot);
}

// bounds of D and its geometry (synchronises)
template <typename T>
reg_status measure_plan(reg_ctx *ctx, const void *D) {
    STCHK(bounds_enqueue<T>(ctx, D, ctx->dpart, kSlotPlanA));
    STCHK(fetch(ctx, kSlotPlanA + 6));
    plan_finish(ctx, D, kSlotPlanA);
    return REG_OK;
}

// departure points from vf (field type), with geometry (synchronises)
template <typename T>
reg_status plan(reg_ctx *ctx, const void *vf, double sign, void *D) {
    STCHK(plan_enqueue<T>(ctx, vf, sign, D, ctx->dpart, kSlotPlanA));
    STCHK(fetch(ctx, kSlotPlanA + 6));
    plan_finish(ctx, D, kSlotPlanA);
    return REG_OK;
}

// public backtrace: v is a velocity-space double vector
template <typename T>
reg_status backtrace_impl(reg_ctx *ctx, const void *v, double sign, void *D) {
    alg_fields(ctx, 3, sizeof(double));
    alg_fields(ctx, 3);
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * ctx->N)));
    return plan<T>(ctx, ctx->vf, sign, D);
}

template <typename T>
reg_status divergence(reg_ctx *ctx, const void *v, void *d) {
    const long N = ctx->N;
    ctx->fft_lines += 3;
    alg_fields(ctx, 6);
    for (int j = 0; j < 3; j++)
        HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<T>(ctx->spec, j, CV<T>(v) + j * N, N, V<T>(d), N, j > 0, 1, ctx->stream)));
    return REG_OK;
}

// grad of nf scalar fields u + k*N into out + k*3N
template <typename T>
reg_status gradient_fields(reg_ctx *ctx, const void *u, int nf, void *out) {
    const long N = ctx->N;
    ctx->fft_lines += 3 * nf;
    alg_fields(ctx, 6.0 * nf);
    for (int j = 0; j < 3; j++)
        HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<T>(ctx->spec, j, CV<T>(u), N, V<T>(out) + j * N, 3 * N, 0, nf, ctx->stream)));
    return REG_OK;
}

// spectral resampling of ncomp field-type fields from src's grid to dst's
// (src's transform buffer, then dst's), on src's stream
template <typename T>
reg_status resample_fields(reg_ctx *src, reg_ctx *dst, int ncomp, const void *in, void *out) {
    hipStream_t st = src->stream;
    // all of it on src's account: the work runs on src's stream
    alg_fft3d(src, ncomp, sizeof(T));
    src->alg_bytes += ncomp * 2.0 * ((double)src->Nh + (double)dst->Nh) * sizeof(T);
    src->alg_bytes += ncomp * ((double)dst->N + 10.0 * (double)dst->Nh) * sizeof(T);
    HIPCHK(src, KL(src, REG_K_FFT3D, (regk::spec_forward<T, T>(src->spec, CV<T>(in), ncomp, 0, st))));
    HIPCHK(src, KL(src, REG_K_SYMBOL, regk::spec_resample<T>(src->spec, dst->spec, ncomp, st)));
    HIPCHK(src, KL(src, REG_K_FFT3D, (regk::spec_inverse<T, T>(dst->spec, V<T>(out), ncomp, st))));
    return REG_OK;
}

// spectral resampling of a velocity-space vector (3 half spectra of complex
// double) from src's grid to dst's: truncation or zero-padding of the modes
inline reg_status resample_vec_hat(reg_ctx *src, const void *xhat, reg_ctx *dst, void *yhat) {
    src->alg_bytes += 6.0 * ((double)src->Nh + (double)dst->Nh) * sizeof(double);
    regk::SpecCtx a = src->spec, b = dst->spec;
    a.H = const_cast<void *>(xhat);
    b.H = yhat;
    HIPCHK(src, KL(src, REG_K_SYMBOL, regk::spec_resample<double>(a, b, 3, src->stream)));
    return REG_OK;
}

// ------------------------------------------- spectral velocity-space vectors
// v, g and the Krylov vectors live on the half spectrum (vec_symbol): the
// regulariser, the preconditioner, the Leray projection and the inner
// products are pointwise there, and only the transport operands (v and the
// matvec direction, in the field type) and the transport result b pass
// through 3D transforms.

// doubles in a spectral velocity vector (also the element count of a PCG
// vector of complex T)
inline long sv_len(const reg_ctx *c) { return 6 * c->Nh; }

// the regulariser 1/2 beta ||lap v||^2 from biharmonic partials in dpart2
inline reg_status reg_term_to_slot(reg_ctx *ctx, int slot) {
    const double N = (double)ctx->N;
    const double scale = 0.5 * ctx->beta * kTwoPi * kTwoPi * kTwoPi / (N * N);
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart2, regk::RED_BLOCKS, scale, ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// sum_k w |k|^4 |v^|^2 partials of a spectral vector into dpart2
inline reg_status biharm_partials(reg_ctx *ctx, const void *vhat) {
    alg_vecs(ctx, 1, sizeof(double));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::vec_dot_partials(ctx->spec, 1, CV<double>(vhat), nullptr, ctx->dpart2,
                                                             regk::RED_BLOCKS, ctx->stream)));
    return REG_OK;
}

// physical double vector -> spectral
inline reg_status to_spec(reg_ctx *ctx, const void *v, void *vhat) {
    ctx->fft3d += 3;
    alg_fft3d(ctx, 3, sizeof(double));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward_to<double, double>(ctx->spec, CV<double>(v), 3, vhat, ctx->stream))));
    return REG_OK;
}

// spectral -> physical double vector (through the scratch spectrum)
inline reg_status from_spec(reg_ctx *ctx, const void *vhat, void *v) {
    ctx->fft3d += 3;
    alg_vecs(ctx, 2, sizeof(double));
    alg_fft3d(ctx, 3, sizeof(double));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::vec_load<double>(ctx->spec, CV<double>(vhat), ctx->H, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse_from<double, double>(ctx->spec, ctx->H, V<double>(v), 3, ctx->stream))));
    return REG_OK;
}

// spectral -> field-type vector for the transport (transform in T)
template <typename T>
reg_status spec_to_field(reg_ctx *ctx, const void *vhat, void *out) {
    ctx->fft3d += 3;
    alg_vecs(ctx, 1, sizeof(double));
    alg_vecs(ctx, 1, sizeof(T));
    alg_fft3d(ctx, 3, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::vec_load<T>(ctx->spec, CV<double>(vhat), ctx->H, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse_from<T, T>(ctx->spec, ctx->H, V<T>(out), 3, ctx->stream))));
    return REG_OK;
}

// the same from a Krylov vector (complex T, the layout of the transform
// buffer), read by the first inverse pass
template <typename T>
reg_status field_from_krylov(reg_ctx *ctx, const void *p, void *out) {
    ctx->fft3d += 3;
    alg_fft3d(ctx, 3, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse_from<T, T>(ctx->spec, ctx->H, V<T>(out), 3, ctx->stream, p))));
    return REG_OK;
}

// out^ = beta |k|^4 x^ + [P] FFT(y), y a field-type vector (transformed in
// T); with dot = 1 (2) also dres[slot] = <x, out> (<out, out>)
template <typename T>
reg_status assemble(reg_ctx *ctx, const void *xhat, const void *y, void *out_hat, int dot = 0, int slot = 0) {
    ctx->fft3d += 3;
    alg_fft3d(ctx, 3, sizeof(T));
    alg_vecs(ctx, out_hat ? 2 : 1, sizeof(double));  // x^ in, out^ out when wanted
    alg_vecs(ctx, 1, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward_to<T, T>(ctx->spec, CV<T>(y), 3, ctx->H, ctx->stream))));
    if (!dot) {
        HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::vec_symbol<T>(ctx->spec, regk::VEC_ASSEMBLE, CV<double>(xhat), ctx->H,
                                                              ctx->beta, ctx->P.isochoric, V<double>(out_hat), ctx->stream)));
        return REG_OK;
    }
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::vec_assemble_dot<T>(ctx->spec, CV<double>(xhat), ctx->H, ctx->beta,
                                                                ctx->P.isochoric, dot, V<double>(out_hat), ctx->dpart,
                                                                regk::RED_BLOCKS, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, h3(ctx) / (double)ctx->N,
                                                            ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// The PCG vectors shat, rhat, phat hold complex T values during a solve
// (see regk::pcg_start).

// PCG set-up of a Newton step (s = 0, r = -g, p = M r) with
// dres[slot] = <r, M r>
template <typename T>
reg_status pcg_start(reg_ctx *ctx, int slot) {
    alg_vecs(ctx, 1, sizeof(double));
    alg_vecs(ctx, 3, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::pcg_start<T>(ctx->spec, CV<double>(ctx->ghat), ctx->beta, ctx->P.isochoric,
                                                         ctx->shat, ctx->rhat, ctx->phat, ctx->dpart,
                                                         regk::RED_BLOCKS, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, h3(ctx) / (double)ctx->N,
                                                            ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// PCG step after a matvec of p whose transformed b~ is still in the
// transform buffer (s += a p, r -= a q) with dres[slot_rr] = <r, r> and
// dres[slot_rz] = <r, M r>
template <typename T>
reg_status pcg_step(reg_ctx *ctx, double a, int slot_rr, int slot_rz) {
    alg_vecs(ctx, 6, sizeof(T));  // p, the b~ transform, s, r in; s, r out
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::pcg_step<T>(ctx->spec, a, ctx->phat, ctx->H, ctx->beta, ctx->P.isochoric,
                                                        ctx->shat, ctx->rhat, ctx->dpart, ctx->dpart2,
                                                        regk::RED_BLOCKS, ctx->stream)));
    const double sc = h3(ctx) / (double)ctx->N;
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, sc, ctx->dres + slot_rr, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart2, regk::RED_BLOCKS, sc, ctx->dres + slot_rz, ctx->stream)));
    return REG_OK;
}

// next PCG direction p = M r + b p
template <typename T>
reg_status pcg_direction(reg_ctx *ctx, double b) {
    alg_vecs(ctx, 3, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::pcg_direction<T>(ctx->spec, ctx->rhat, b, ctx->beta, ctx->P.isochoric,
                                                             ctx->phat, ctx->stream)));
    return REG_OK;
}

// dres[slot] = <a, b> for a velocity vector a and a PCG vector b
template <typename T>
reg_status krylov_dot(reg_ctx *ctx, const void *a, const void *b, int slot) {
    alg_vecs(ctx, 1, sizeof(double));
    alg_vecs(ctx, 1, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::krylov_dot_partials<T>(ctx->spec, CV<double>(a), b, ctx->dpart,
                                                                   regk::RED_BLOCKS, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, h3(ctx) / (double)ctx->N,
                                                            ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// out = x + a y for velocity vectors x, out and a PCG vector y
template <typename T>
reg_status krylov_axpy(reg_ctx *ctx, const void *x, double a, const void *y, void *out) {
    alg_vecs(ctx, 2, sizeof(double));
    alg_vecs(ctx, 1, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::krylov_axpy<T>(ctx->spec, CV<double>(x), a, y, V<double>(out), ctx->stream)));
    return REG_OK;
}

// dres[slot] = <p, beta |k|^4 p + [P] FFT(y)> for the PCG vector p, y a
// field-type vector (FFT(y) stays in the transform buffer)
template <typename T>
reg_status curvature(reg_ctx *ctx, const void *p, const void *y, int slot) {
    ctx->fft3d += 3;
    alg_fft3d(ctx, 3, sizeof(T));
    alg_vecs(ctx, 2, sizeof(T));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward_to<T, T>(ctx->spec, CV<T>(y), 3, ctx->H, ctx->stream))));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::krylov_curvature<T>(ctx->spec, p, ctx->H, ctx->beta, ctx->P.isochoric,
                                                                ctx->dpart, regk::RED_BLOCKS, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, h3(ctx) / (double)ctx->N,
                                                            ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// z^ = M r^: inverse biharmonic (identity at k = 0), then P when isochoric
inline reg_status precond_hat(reg_ctx *ctx, const void *rhat, void *zhat) {
    alg_vecs(ctx, 2, sizeof(double));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::vec_symbol<double>(ctx->spec, regk::VEC_PRECOND, CV<double>(rhat), nullptr,
                                                               ctx->beta, ctx->P.isochoric, V<double>(zhat), ctx->stream)));
    return REG_OK;
}

inline reg_status leray_hat(reg_ctx *ctx, void *vhat) {
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::vec_symbol<double>(ctx->spec, regk::VEC_LERAY, CV<double>(vhat), nullptr,
                                                               0.0, 1, V<double>(vhat), ctx->stream)));
    return REG_OK;
}

// mismatch^2 numerator (slot 1) and regulariser (slot 2) of the history in
// hist at the spectral velocity vhat (reg_done: its biharmonic partials are
// already in dpart2)
template <typename T>
reg_status objective_slots(reg_ctx *ctx, const void *hist, const void *vhat, bool reg_done) {
    const long N = ctx->N;
    STCHK(reduce<T>(ctx, V<T>(const_cast<void *>(hist)) + (long)ctx->P.nt * N, ctx->rhoR, N, 1, h3(ctx), 1));
    if (!reg_done) STCHK(biharm_partials(ctx, vhat));
    return reg_term_to_slot(ctx, 2);
}

inline void scalars_to_J(reg_ctx *ctx, double *J, double *mis) {
    const double dd = ctx->hres[1];
    if (J) *J = 0.5 * dd + ctx->hres[2];
    if (mis) *mis = ctx->normTR2 > 0 ? std::sqrt(dd / ctx->normTR2) : 0.0;
}

// The map y1 = x + u of v (eq. (1)): u transported like the state,
// u^{n+1} = u^n(X) + h D, then det(I + grad u) by spectral derivatives, its
// minimum and maximum (synchronises). u_out may be null.
template <typename T>
reg_status deformation_impl(reg_ctx *ctx, const void *v, void *u_out, double *dmin, double *dmax) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * N)));
    STCHK(plan<T>(ctx, ctx->vf, +1.0, ctx->Dt));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_fill<T>(3 * N, 0.0, V<T>(ctx->u0), ctx->stream)));
    void *ub[2] = {ctx->u0, ctx->u1};
    int cur = 0;
    for (int k = 0; k < nt; k++) {
        HIPCHK(ctx, KL(ctx, REG_K_DEFORM, regk::launch_deform_step<T>(ctx->g, V<T>(ub[cur]), CV<T>(ctx->Dt), V<T>(ub[1 - cur]),
                                                ctx->stream)));
        cur = 1 - cur;
    }
    ctx->interps += 3 * nt;
    alg_fields(ctx, 3 + 9.0 * nt + 18 + 9);  // zero u, the steps, the nine derivatives, det
    // du[a*3+b] = d_b u_a
    for (int b = 0; b < 3; b++)
        HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<T>(ctx->spec, b, V<T>(ub[cur]), N, V<T>(ctx->du) + b * N, 3 * N, 0, 3,
                                        ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_det_partials<T>(V<T>(ctx->du), N, ctx->dpart, ctx->dpart2, (T *)nullptr, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize_minmax(ctx->dpart, ctx->dpart2, regk::RED_BLOCKS, ctx->dres, ctx->stream)));
    if (u_out) HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(3 * N, V<T>(ub[cur]), V<T>(u_out), ctx->stream)));
    STCHK(fetch(ctx, 2));
    *dmin = ctx->hres[0];
    *dmax = ctx->hres[1];
    return REG_OK;
}

using clk = std::chrono::steady_clock;
inline double secs(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }


}  // namespace regc
