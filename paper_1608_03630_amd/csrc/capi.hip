// C ABI of libreg (declared in include/reg.h): the context over a
// caller-owned workspace, the transport solves, reduced gradient, Gauss-Newton
// Hessian matvec and preconditioner, and the Gauss-Newton-Krylov driver of
// section III-A of the paper. Host code only orchestrates: every grid-sized
// operation runs in the kernels of interp.hip, fft.hip and blas.hip; the host
// reads back double-precision scalars (inner products, objective, norms)
// where the Newton-Krylov iteration branches on them.
//
// Precision: image-space fields (images, state and adjoint histories, grad
// rho, departure points, b) use the field type T of params.prec; the
// velocity-space vectors (v, g, the PCG vectors) are always double and the 3D
// spectral operators that act on them (lap^2, its inverse, P, the gradient
// and matvec assembly) run in double. The H2 regulariser multiplies the
// representation error of v by |k|^4 (up to (n sqrt(3)/2)^4, about 2.4e9 on
// a 256^3 grid), which single precision cannot absorb; the transport, whose
// data are smooth images, runs in T.
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

namespace {

constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr size_t kAlign = 256;
constexpr int kSlots = 16;  // device result slots (doubles)

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool fft_friendly(int n) {
    if (n < 8 || n > 1024 || (n & 1)) return false;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
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

}  // namespace

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
    void *lamh;        // adjoint levels lam^0..lam^nt
    void *gam, *gam2;  // Heun factor of the adjoint source (cached plan, scratch plan)
    void *vf, *vtf;                                            // velocity copies in the field type
    void *vcur, *g_, *sdir, *r, *z, *p, *q, *vtrial;          // velocity space, double
    void *u0, *u1, *du, *H;
    void *tw32[3], *tw64[3];
    double *dpart, *dpart2, *dres;
    double *hres = nullptr;  // pinned host mirror of dres

    // profiler: event pairs around launches, resolved after stream syncs
    struct ProfRec {
        hipEvent_t a, b;
        int kind;
    };
    bool prof_on = false;
    std::vector<hipEvent_t> ev_free;
    std::vector<ProfRec> ev_pending;
    double prof_ms[REG_K_COUNT] = {0};
    int64_t prof_n[REG_K_COUNT] = {0};

    // tile geometry of the LDS-staged gathers, per displacement buffer
    struct PlanGeom {
        const void *D = nullptr;
        bool tiled = false;
        regk::TileGeom tg{};
    };
    PlanGeom geoms[6];

    bool have_images = false;
    bool have_state = false;  // plans, history, grad rho and div v at vcur
    double normTR2 = 0;       // <rho_T - rho_R, rho_T - rho_R>
    long interps = 0;
    std::string err;
};

namespace {

reg_status fail(reg_ctx *ctx, reg_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return st;
}

reg_status hipfail(reg_ctx *ctx, hipError_t e, const char *what) {
    return fail(ctx, REG_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr)                                         \
    do {                                                          \
        hipError_t e_ = (expr);                                   \
        if (e_ != hipSuccess) return hipfail((ctx), e_, #expr);  \
    } while (0)

// Adds the elapsed times of completed event pairs to the counters (the
// stream has been synchronised by the caller).
void prof_resolve(reg_ctx *ctx) {
    for (auto &r : ctx->ev_pending) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
            ctx->prof_ms[r.kind] += ms;
            ctx->prof_n[r.kind] += 1;
        } else {
            (void)hipGetLastError();
        }
        ctx->ev_free.push_back(r.a);
        ctx->ev_free.push_back(r.b);
    }
    ctx->ev_pending.clear();
}

hipEvent_t take_event(reg_ctx *ctx) {
    if (ctx->ev_free.empty()) {
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        return e;
    }
    hipEvent_t e = ctx->ev_free.back();
    ctx->ev_free.pop_back();
    return e;
}

// Runs one launcher; with profiling on, brackets it with two events.
template <class F>
hipError_t timed(reg_ctx *ctx, int kind, F &&launch) {
    if (!ctx->prof_on) return launch();
    if (ctx->ev_pending.size() >= 8192) {
        hipError_t e = hipStreamSynchronize(ctx->stream);
        if (e != hipSuccess) return e;
        prof_resolve(ctx);
    }
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return launch();
    hipError_t e = hipEventRecord(a, ctx->stream);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, ctx->stream);
    if (e != hipSuccess) return e;
    ctx->ev_pending.push_back({a, b, kind});
    return hipSuccess;
}

#define KL(ctx, kind, expr) timed((ctx), (kind), [&]() { return (expr); })

#define STCHK(expr)                     \
    do {                                \
        reg_status s_ = (expr);         \
        if (s_ != REG_OK) return s_;    \
    } while (0)

reg_status check_params(const reg_params *p, std::string *why) {
    if (!p) {
        *why = "params is NULL";
        return REG_EINVAL;
    }
    for (int j = 0; j < 3; j++)
        if (!fft_friendly(p->n[j])) {
            *why = "grid size n[" + std::to_string(j) + "] = " + std::to_string(p->n[j]) +
                   " must be even, 2^a 3^b and in [8, 1024]";
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
    return REG_OK;
}

// Lays out the workspace of a context (ctx == nullptr: size only).
size_t layout(const reg_params *p, char *base, reg_ctx *ctx) {
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
    c->grho = L.take(E * 3 * N * nt1);
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
    c->gam = L.take(E * N);
    c->gam2 = L.take(E * N);
    c->bvec = L.take(E * 3 * N);
    c->vf = L.take(E * 3 * N);
    c->vtf = L.take(E * 3 * N);
    const size_t D8 = sizeof(double);
    c->vcur = L.take(D8 * 3 * N);
    c->g_ = L.take(D8 * 3 * N);
    c->sdir = L.take(D8 * 3 * N);
    c->r = L.take(D8 * 3 * N);
    c->z = L.take(D8 * 3 * N);
    c->p = L.take(D8 * 3 * N);
    c->q = L.take(D8 * 3 * N);
    c->vtrial = L.take(D8 * 3 * N);
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

bool is_device_ptr(const void *ptr) {
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

double h3(const reg_ctx *c) { return (kTwoPi / c->g.n1) * (kTwoPi / c->g.n2) * (kTwoPi / c->g.n3); }

const regk::TileGeom *geom_of(const reg_ctx *ctx, const void *D) {
    for (const auto &g : ctx->geoms)
        if (g.D == D) return g.tiled ? &g.tg : nullptr;
    return nullptr;
}

void set_geom(reg_ctx *ctx, const void *D, bool tiled, const regk::TileGeom &tg) {
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

// reads kSlots doubles back (synchronises)
reg_status fetch(reg_ctx *ctx, int nslots) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * nslots, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (!ctx->ev_pending.empty()) prof_resolve(ctx);
    return REG_OK;
}

// dres[slot] = scale * reduction
template <typename T>
reg_status reduce(reg_ctx *ctx, const void *a, const void *b, long n, int mode, double scale, int slot) {
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_dot_partials<T>(CV<T>(a), CV<T>(b ? b : a), n, mode, ctx->dpart, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart, regk::RED_BLOCKS, scale, ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

template <typename T>
reg_status plan(reg_ctx *ctx, const void *v, double sign, void *D);

// public backtrace: v is a velocity-space double vector
template <typename T>
reg_status backtrace_impl(reg_ctx *ctx, const void *v, double sign, void *D) {
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * ctx->N)));
    return plan<T>(ctx, ctx->vf, sign, D);
}

// floor bounds of D over the grid -> tile geometry of the gathers that use D
// (synchronises)
template <typename T>
reg_status measure_plan(reg_ctx *ctx, const void *D) {
    const int nb = regk::RED_BLOCKS / 6;
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_floor_bounds<T>(ctx->g, CV<T>(D), ctx->dpart, nb, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize_bounds(ctx->dpart, nb, ctx->dres + 8, ctx->stream)));
    STCHK(fetch(ctx, 14));
    double fmin[3], fmax[3];
    for (int j = 0; j < 3; j++) {
        fmin[j] = ctx->hres[8 + 2 * j];
        fmax[j] = ctx->hres[8 + 2 * j + 1];
    }
    regk::TileGeom tg{};
    const bool ok = regk::tile_geom(fmin, fmax, sizeof(T), &tg);
    set_geom(ctx, D, ok, tg);
    return REG_OK;
}

// departure points from vf (field type)
template <typename T>
reg_status plan(reg_ctx *ctx, const void *v, double sign, void *D) {
    HIPCHK(ctx, KL(ctx, REG_K_BACKTRACE, regk::launch_backtrace<T>(ctx->g, CV<T>(v), sign / ctx->P.nt, V<T>(D), ctx->stream)));
    ctx->interps += 3;
    return measure_plan<T>(ctx, D);
}

// hist[0] = rho0, hist[n+1] = hist[n](X)
template <typename T>
reg_status state_solve(reg_ctx *ctx, const void *Df, const void *rho0, void *hist) {
    const long N = ctx->N;
    if (rho0 != hist) HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(N, CV<T>(rho0), V<T>(hist), ctx->stream)));
    for (int k = 0; k < ctx->P.nt; k++)
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, V<T>(hist) + k * N, CV<T>(Df), V<T>(hist) + (k + 1) * N,
                                           ctx->stream, geom_of(ctx, Df))));
    ctx->interps += ctx->P.nt;
    return REG_OK;
}

// d = div v by line FFTs (three accumulating derivative passes)
template <typename T>
reg_status divergence(reg_ctx *ctx, const void *v, void *d) {
    const long N = ctx->N;
    for (int j = 0; j < 3; j++)
        HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<T>(ctx->spec, j, CV<T>(v) + j * N, N, V<T>(d), N, j > 0, 1, ctx->stream)));
    return REG_OK;
}

// grad of nf scalar fields u + k*N into out + k*3N
template <typename T>
reg_status gradient_fields(reg_ctx *ctx, const void *u, int nf, void *out) {
    const long N = ctx->N;
    for (int j = 0; j < 3; j++)
        HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<T>(ctx->spec, j, CV<T>(u), N, V<T>(out) + j * N, 3 * N, 0, nf, ctx->stream)));
    return REG_OK;
}

// out = IFFT(beta |k|^4 x^ + [P] y^); also leaves sum w |k|^4 |x^|^2 partials
// in dpart2 when want_reg
// (x and out are velocity-space doubles, y is a field-type vector; the
// transforms run in double)
template <typename T>
reg_status assemble(reg_ctx *ctx, const void *x, const void *y, void *out, bool want_reg) {
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<double, double>(ctx->spec, CV<double>(x), 3, 0, ctx->stream))));
    if (want_reg) HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_biharm_norm_partials<double>(ctx->spec, ctx->dpart2, regk::RED_BLOCKS, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<T, double>(ctx->spec, CV<T>(y), 3, 3, ctx->stream))));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_symbol<double>(ctx->spec, regk::SYM_ASSEMBLE, ctx->beta, 3, ctx->P.isochoric, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse<double, double>(ctx->spec, V<double>(out), 3, ctx->stream))));
    return REG_OK;
}

// the regulariser 1/2 beta ||lap v||^2 from biharmonic partials in dpart2
reg_status reg_term_to_slot(reg_ctx *ctx, int slot) {
    const double N = (double)ctx->N;
    const double scale = 0.5 * ctx->beta * kTwoPi * kTwoPi * kTwoPi / (N * N);
    HIPCHK(ctx, KL(ctx, REG_K_REDUCE, regk::launch_finalize(ctx->dpart2, regk::RED_BLOCKS, scale, ctx->dres + slot, ctx->stream)));
    return REG_OK;
}

// v is a velocity-space double vector
reg_status regulariser_of(reg_ctx *ctx, const void *v, int slot) {
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<double, double>(ctx->spec, CV<double>(v), 3, 0, ctx->stream))));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_biharm_norm_partials<double>(ctx->spec, ctx->dpart2, regk::RED_BLOCKS, ctx->stream)));
    return reg_term_to_slot(ctx, slot);
}

// Backward adjoint-type sweep: lamh[nt] holds lam^nt; writes lam^n for
// n = nt-1..0, then b = sum_n w_n lam^n grad rho^n in one pass.
template <typename T>
reg_status adjoint_sweep(reg_ctx *ctx, const void *Da, const void *gam, void *b) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    for (int k = nt - 1; k >= 0; k--)
        HIPCHK(ctx, KL(ctx, REG_K_ADJOINT, regk::launch_adjoint_step<T>(ctx->g, V<T>(ctx->lamh) + (long)(k + 1) * N, CV<T>(Da),
                                                 CV<T>(gam), V<T>(ctx->lamh) + (long)k * N, ctx->stream,
                                                 geom_of(ctx, Da))));
    ctx->interps += nt;
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_b_assemble<T>(N, nt, CV<T>(ctx->lamh), CV<T>(ctx->grho), V<T>(b), ctx->stream)));
    return REG_OK;
}

// plan for -v, grad rho^n and div v: completes the cached state at vcur
// (vf holds vcur in the field type)
template <typename T>
reg_status complete_state(reg_ctx *ctx) {
    STCHK(plan<T>(ctx, ctx->vf, -1.0, ctx->Da));
    STCHK(gradient_fields<T>(ctx, ctx->histA, ctx->P.nt + 1, ctx->grho));
    if (!ctx->P.isochoric) {
        STCHK(divergence<T>(ctx, ctx->vf, ctx->c));
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, CV<T>(ctx->c), CV<T>(ctx->Da), V<T>(ctx->cX), ctx->stream,
                                                                 geom_of(ctx, ctx->Da))));
        ctx->interps += 1;
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_gamma<T>(ctx->N, CV<T>(ctx->c), CV<T>(ctx->cX), V<T>(ctx->gam),
                                                                1.0 / ctx->P.nt, ctx->stream)));
    }
    ctx->have_state = true;
    return REG_OK;
}

// J (slot 0), mismatch^2 numerator (slot 1) of the history in hist at v
template <typename T>
reg_status objective_slots(reg_ctx *ctx, const void *hist, const void *v, bool reg_done) {
    const long N = ctx->N;
    STCHK(reduce<T>(ctx, V<T>(const_cast<void *>(hist)) + (long)ctx->P.nt * N, ctx->rhoR, N, 1, h3(ctx), 1));
    if (!reg_done) STCHK(regulariser_of(ctx, v, 2));
    else STCHK(reg_term_to_slot(ctx, 2));
    return REG_OK;
}

void scalars_to_J(reg_ctx *ctx, double *J, double *mis) {
    const double dd = ctx->hres[1];
    if (J) *J = 0.5 * dd + ctx->hres[2];
    if (mis) *mis = ctx->normTR2 > 0 ? std::sqrt(dd / ctx->normTR2) : 0.0;
}

// gradient at v with the state recomputed (or reused when reuse_trial: histB
// and Dt already hold the plan and state of v)
template <typename T>
reg_status gradient_impl(reg_ctx *ctx, const void *v, void *g, double *J, double *mis, double *gnorm,
                         bool reuse_trial) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    if (v != ctx->vcur) HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(3 * N, CV<double>(v), V<double>(ctx->vcur), ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, ctx->vcur, ctx->vf, 3 * N)));
    if (reuse_trial) {
        std::swap(ctx->histA, ctx->histB);
        std::swap(ctx->Df, ctx->Dt);
    } else {
        STCHK(plan<T>(ctx, ctx->vf, +1.0, ctx->Df));
        STCHK(state_solve<T>(ctx, ctx->Df, ctx->rhoT, ctx->histA));
    }
    STCHK(complete_state<T>(ctx));
    // adjoint from lam(1) = rho_R - rho(1), b = sum w_n lam^n grad rho^n
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_adjoint_init<T>(N, CV<T>(ctx->rhoR), V<T>(ctx->histA) + (long)nt * N,
                                                                   V<T>(ctx->lamh) + (long)nt * N, ctx->stream)));
    STCHK(adjoint_sweep<T>(ctx, ctx->Da, ctx->P.isochoric ? nullptr : ctx->gam, ctx->bvec));
    STCHK(assemble<T>(ctx, ctx->vcur, ctx->bvec, g, true));
    STCHK(objective_slots<T>(ctx, ctx->histA, ctx->vcur, true));
    STCHK(reduce<double>(ctx, g, nullptr, 3 * N, 2, h3(ctx), 3));
    STCHK(fetch(ctx, 4));
    scalars_to_J(ctx, J, mis);
    if (gnorm) *gnorm = std::sqrt(ctx->hres[3]);
    if (!std::isfinite(ctx->hres[1]) || !std::isfinite(ctx->hres[2]) || !std::isfinite(ctx->hres[3]))
        return fail(ctx, REG_ENONFINITE, "non-finite objective or gradient");
    return REG_OK;
}

template <typename T>
reg_status matvec_impl(reg_ctx *ctx, const void *vt, void *Hvt) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    const double dt = 1.0 / nt;
    // incremental state through q^n = rho~^n - dt/2 vt.grad rho^n
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, vt, ctx->vtf, 3 * N)));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_incstate_init<T>(ctx->g, CV<T>(ctx->vtf), V<T>(ctx->grho), V<T>(ctx->lam[1]), -0.5 * dt,
                                              ctx->stream)));
    int cur = 1;
    for (int k = 0; k < nt; k++) {
        const int last = (k == nt - 1);
        T *dst = last ? V<T>(ctx->lamh) + (long)nt * N : V<T>(ctx->lam[1 - cur]);
        HIPCHK(ctx, KL(ctx, REG_K_INCSTATE, regk::launch_incstate_step<T>(ctx->g, V<T>(ctx->lam[cur]), CV<T>(ctx->Df), CV<T>(ctx->vtf),
                                                  V<T>(ctx->grho) + (long)(k + 1) * 3 * N, dst,
                                                  last ? -0.5 * dt : -dt, last, ctx->stream, geom_of(ctx, ctx->Df))));
        cur = 1 - cur;
    }
    ctx->interps += nt;
    // lam~(1) = -rho~(1) now sits in lamh[nt]
    STCHK(adjoint_sweep<T>(ctx, ctx->Da, ctx->P.isochoric ? nullptr : ctx->gam, ctx->bvec));
    STCHK(assemble<T>(ctx, vt, ctx->bvec, Hvt, false));
    return REG_OK;
}

// r and z are velocity-space doubles
reg_status precond_impl(reg_ctx *ctx, const void *r, void *z) {
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<double, double>(ctx->spec, CV<double>(r), 3, 0, ctx->stream))));
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_symbol<double>(ctx->spec, regk::SYM_PRECOND, ctx->beta, 3, ctx->P.isochoric, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse<double, double>(ctx->spec, V<double>(z), 3, ctx->stream))));
    return REG_OK;
}

// J and mismatch of a trial velocity: plan into Dt, state into histB
template <typename T>
reg_status trial_objective(reg_ctx *ctx, const void *v, double *J, double *mis) {
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * ctx->N)));
    STCHK(plan<T>(ctx, ctx->vf, +1.0, ctx->Dt));
    STCHK(state_solve<T>(ctx, ctx->Dt, ctx->rhoT, ctx->histB));
    STCHK(objective_slots<T>(ctx, ctx->histB, v, false));
    STCHK(fetch(ctx, 3));
    scalars_to_J(ctx, J, mis);
    if (!std::isfinite(*J)) return fail(ctx, REG_ENONFINITE, "non-finite objective");
    return REG_OK;
}

// inner product of two velocity-space vectors
reg_status dot3(reg_ctx *ctx, const void *a, const void *b, double *out) {
    STCHK(reduce<double>(ctx, a, b, 3 * ctx->N, 0, h3(ctx), 0));
    STCHK(fetch(ctx, 1));
    *out = ctx->hres[0];
    return REG_OK;
}

using clk = std::chrono::steady_clock;
double secs(clk::time_point a) { return std::chrono::duration<double>(clk::now() - a).count(); }

template <typename T>
reg_status solve_impl(reg_ctx *ctx, void *v, reg_report *rep) {
    const reg_params &P = ctx->P;
    const long N3 = 3 * ctx->N;
    auto t0 = clk::now();
    const long interps0 = ctx->interps;
    if (P.isochoric) {
        HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<double, double>(ctx->spec, CV<double>(v), 3, 0, ctx->stream))));
        HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_symbol<double>(ctx->spec, regk::SYM_LERAY, 0.0, 3, 1, ctx->stream)));
        HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse<double, double>(ctx->spec, V<double>(v), 3, ctx->stream))));
    }
    const double beta_final = P.beta_final > 0 ? P.beta_final : P.beta;
    const double factor = (P.beta_factor > 0 && P.beta_factor < 1) ? P.beta_factor : 0.1;
    double beta = P.beta;
    int it = 0;
    double J = 0, mis = 0, gnorm = 0, g0 = 0;
    reg_status status = REG_OK;
    bool done = false;
    while (!done) {
        ctx->beta = beta;
        auto tg = clk::now();
        STCHK(gradient_impl<T>(ctx, v, ctx->g_, &J, &mis, &gnorm, false));
        rep->seconds_gradient += secs(tg);
        rep->gradients++;
        g0 = gnorm;
        rep->stop_reason = 2;
        for (int k = 0; k < P.max_newton; k++) {
            if (gnorm <= P.gtol * g0) {
                rep->stop_reason = 0;
                break;
            }
            if (P.mismatch_tol > 0 && mis <= P.mismatch_tol) {
                rep->stop_reason = 1;
                break;
            }
            const double ratio = g0 > 0 ? gnorm / g0 : 0.0;
            double eta = P.forcing == 1 ? std::sqrt(ratio) : ratio;
            if (eta > 0.5) eta = 0.5;
            // truncated PCG on H s = -g
            HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_fill<double>(N3, 0.0, V<double>(ctx->sdir), ctx->stream)));
            HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_axpby<double>(N3, -1.0, CV<double>(ctx->g_), 0.0, V<double>(ctx->r), ctx->stream)));
            auto tp = clk::now();
            STCHK(precond_impl(ctx, ctx->r, ctx->z));
            rep->seconds_precond += secs(tp);
            HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(N3, CV<double>(ctx->z), V<double>(ctx->p), ctx->stream)));
            double rz;
            STCHK(dot3(ctx, ctx->r, ctx->z, &rz));
            int iters = 0;
            for (int i = 0; i < P.max_pcg; i++) {
                auto tm = clk::now();
                STCHK(matvec_impl<T>(ctx, ctx->p, ctx->q));
                double kappa;
                STCHK(dot3(ctx, ctx->p, ctx->q, &kappa));
                rep->seconds_matvec += secs(tm);
                rep->matvecs++;
                iters = i + 1;
                if (!std::isfinite(kappa)) return fail(ctx, REG_ENONFINITE, "non-finite curvature in PCG");
                if (kappa <= 0) {
                    if (i == 0) HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(N3, CV<double>(ctx->z), V<double>(ctx->sdir), ctx->stream)));
                    break;
                }
                const double a = rz / kappa;
                HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_cg_update<double>(N3, a, CV<double>(ctx->p), CV<double>(ctx->q), V<double>(ctx->sdir),
                                                      V<double>(ctx->r), ctx->stream)));
                double rr;
                STCHK(dot3(ctx, ctx->r, ctx->r, &rr));
                if (std::sqrt(rr) <= eta * gnorm) break;
                tp = clk::now();
                STCHK(precond_impl(ctx, ctx->r, ctx->z));
                rep->seconds_precond += secs(tp);
                double rz1;
                STCHK(dot3(ctx, ctx->r, ctx->z, &rz1));
                HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_xpay<double>(N3, CV<double>(ctx->z), rz1 / rz, CV<double>(ctx->p), V<double>(ctx->p),
                                                 ctx->stream)));
                rz = rz1;
            }
            // Armijo backtracking
            double d;
            STCHK(dot3(ctx, ctx->g_, ctx->sdir, &d));
            double alpha = 1.0, Jt = 0, mist = 0;
            int trials = 0;
            bool accepted = false;
            auto to = clk::now();
            for (int l = 0; l < P.max_ls; l++) {
                trials++;
                HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_xpay<double>(N3, CV<double>(v), alpha, CV<double>(ctx->sdir), V<double>(ctx->vtrial),
                                                 ctx->stream)));
                STCHK(trial_objective<T>(ctx, ctx->vtrial, &Jt, &mist));
                rep->objectives++;
                if (Jt <= J + P.armijo_c1 * alpha * d) {
                    accepted = true;
                    break;
                }
                alpha *= 0.5;
            }
            rep->seconds_objective += secs(to);
            if (!accepted) {
                status = fail(ctx, REG_ELINESEARCH, "Armijo line search found no acceptable step");
                done = true;
                break;
            }
            HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(N3, CV<double>(ctx->vtrial), V<double>(v), ctx->stream)));
            tg = clk::now();
            STCHK(gradient_impl<T>(ctx, v, ctx->g_, &J, &mis, &gnorm, true));
            rep->seconds_gradient += secs(tg);
            rep->gradients++;
            if (it < REG_MAXIT) {
                rep->J[it] = J;
                rep->mismatch[it] = mis;
                rep->grel[it] = g0 > 0 ? gnorm / g0 : 0;
                rep->alpha[it] = alpha;
                rep->beta[it] = beta;
                rep->pcg_iters[it] = iters;
                rep->ls_trials[it] = trials;
            }
            it++;
            rep->stop_reason = 2;
        }
        if (done) break;
        if (rep->stop_reason == 2) {
            if (gnorm <= P.gtol * g0) rep->stop_reason = 0;
            if (P.mismatch_tol > 0 && mis <= P.mismatch_tol) rep->stop_reason = 1;
        }
        if (rep->stop_reason == 1 || beta <= beta_final * (1 + 1e-12)) done = true;
        else {
            beta *= factor;
            if (beta < beta_final) beta = beta_final;
        }
    }
    ctx->beta = P.beta;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    rep->status = status;
    rep->n_iter = it;
    rep->final_J = J;
    rep->final_mismatch = mis;
    rep->final_grel = g0 > 0 ? gnorm / g0 : 0;
    rep->interps = ctx->interps - interps0;
    rep->seconds_total = secs(t0);
    return status;
}

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

template <typename T>
reg_status transport_forward_impl(reg_ctx *ctx, const void *v, const void *rho0, void *rho1) {
    const long N = ctx->N;
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * N)));
    STCHK(plan<T>(ctx, ctx->vf, +1.0, ctx->Dt));
    // ping-pong between two slices of the scratch history, last step into rho1
    const T *src = CV<T>(rho0);
    for (int k = 0; k < ctx->P.nt; k++) {
        T *dst = (k == ctx->P.nt - 1) ? V<T>(rho1) : V<T>(ctx->histB) + (long)(k & 1) * N;
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, src, CV<T>(ctx->Dt), dst, ctx->stream, geom_of(ctx, ctx->Dt))));
        src = dst;
    }
    ctx->interps += ctx->P.nt;
    return REG_OK;
}

template <typename T>
reg_status transport_adjoint_impl(reg_ctx *ctx, const void *v, const void *lam1, void *lam0) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, v, ctx->vf, 3 * N)));
    STCHK(plan<T>(ctx, ctx->vf, -1.0, ctx->Dt));
    const bool src = !ctx->P.isochoric;
    if (src) {
        STCHK(divergence<T>(ctx, ctx->vf, ctx->c2));
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, CV<T>(ctx->c2), CV<T>(ctx->Dt), V<T>(ctx->cX2), ctx->stream, geom_of(ctx, ctx->Dt))));
        ctx->interps += 1;
    }
    if (src)
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_gamma<T>(N, CV<T>(ctx->c2), CV<T>(ctx->cX2), V<T>(ctx->gam2), 1.0 / nt,
                                                                ctx->stream)));
    const T *in = CV<T>(lam1);
    for (int k = 0; k < nt; k++) {
        T *out = (k == nt - 1) ? V<T>(lam0) : V<T>(ctx->histB) + (long)(k & 1) * N;
        HIPCHK(ctx, KL(ctx, REG_K_ADJOINT, regk::launch_adjoint_step<T>(ctx->g, in, CV<T>(ctx->Dt), src ? CV<T>(ctx->gam2) : nullptr,
                                                                        out, ctx->stream, geom_of(ctx, ctx->Dt))));
        in = out;
    }
    ctx->interps += nt;
    return REG_OK;
}

template <typename T>
reg_status spectral_impl(reg_ctx *ctx, int op, double scale, int ncomp, const void *v, void *out) {
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<T, T>(ctx->spec, CV<T>(v), ncomp, 0, ctx->stream))));
    int sym = op == 0 ? regk::SYM_BIHARM : op == 1 ? regk::SYM_INVBIHARM : op == 2 ? regk::SYM_GAUSS : regk::SYM_LERAY;
    HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_symbol<T>(ctx->spec, sym, scale, ncomp, 1, ctx->stream)));
    HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse<T, T>(ctx->spec, V<T>(out), ncomp, ctx->stream))));
    return REG_OK;
}

}  // namespace

// ====================================================================== ABI

#define DISPATCH(ctx, fn, ...) ((ctx)->P.prec ? fn<double>(__VA_ARGS__) : fn<float>(__VA_ARGS__))

#define CTX_OK(ctx)                                   \
    do {                                              \
        if (!(ctx)) return REG_EINVAL;                \
        (ctx)->err.clear();                           \
    } while (0)

extern "C" {

reg_status reg_default_params(reg_params *p) {
    if (!p) return REG_EINVAL;
    std::memset(p, 0, sizeof(*p));
    p->n[0] = p->n[1] = p->n[2] = 64;
    p->nt = 4;
    p->beta = 1e-2;
    p->beta_final = 0.0;
    p->beta_factor = 0.1;
    p->isochoric = 0;
    p->prec = 0;
    p->gtol = 1e-2;
    p->mismatch_tol = 0.0;
    p->max_newton = 50;
    p->max_pcg = 100;
    p->max_ls = 20;
    p->forcing = 0;
    p->armijo_c1 = 1e-4;
    return REG_OK;
}

reg_status reg_workspace_size(const reg_params *p, size_t *bytes) {
    std::string why;
    if (check_params(p, &why) != REG_OK || !bytes) return REG_EINVAL;
    *bytes = layout(p, nullptr, nullptr);
    return REG_OK;
}

reg_status reg_create(const reg_params *p, void *workspace, size_t bytes, void *hip_stream, reg_ctx **out) {
    if (!out) return REG_EINVAL;
    *out = nullptr;
    std::string why;
    if (check_params(p, &why) != REG_OK) {
        std::fprintf(stderr, "reg_create: %s\n", why.c_str());
        return REG_EINVAL;
    }
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0) return REG_EINVAL;
    if (bytes < layout(p, nullptr, nullptr)) return REG_ENOMEM;
    if (!is_device_ptr(workspace)) return REG_EINVAL;
    reg_ctx *ctx = new (std::nothrow) reg_ctx();
    if (!ctx) return REG_ENOMEM;
    ctx->P = *p;
    ctx->beta = p->beta;
    ctx->stream = (hipStream_t)hip_stream;
    (void)hipGetDevice(&ctx->device);
    ctx->g = Grid{p->n[0], p->n[1], p->n[2]};
    ctx->N = ctx->g.N();
    ctx->Nh = ctx->g.Nh();
    ctx->esz = p->prec ? 8 : 4;
    layout(p, (char *)workspace, ctx);
    if (hipHostMalloc((void **)&ctx->hres, sizeof(double) * kSlots, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete ctx;
        return REG_EHIP;
    }
    ctx->spec.g = ctx->g;
    ctx->spec.H = ctx->H;
    for (int j = 0; j < 3; j++) {
        regk::make_plan(p->n[j], &ctx->spec.plan[j]);
        ctx->spec.tw[0][j] = ctx->tw32[j];
        ctx->spec.tw[1][j] = ctx->tw64[j];
        const int n = p->n[j];
        // twiddles exp(-2 pi i m / n), computed in double
        std::vector<double> b64(2 * n);
        std::vector<float> b32(2 * n);
        for (int m = 0; m < n; m++) {
            b64[2 * m] = std::cos(kTwoPi * m / n);
            b64[2 * m + 1] = -std::sin(kTwoPi * m / n);
            b32[2 * m] = (float)b64[2 * m];
            b32[2 * m + 1] = (float)b64[2 * m + 1];
        }
        if (hipMemcpy(ctx->tw64[j], b64.data(), sizeof(double) * 2 * n, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->tw32[j], b32.data(), sizeof(float) * 2 * n, hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(ctx->hres);
            delete ctx;
            return REG_EHIP;
        }
    }
    *out = ctx;
    return REG_OK;
}

reg_status reg_destroy(reg_ctx *ctx) {
    if (!ctx) return REG_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    prof_resolve(ctx);
    for (hipEvent_t e : ctx->ev_free) (void)hipEventDestroy(e);
    if (ctx->hres) (void)hipHostFree(ctx->hres);
    delete ctx;
    return REG_OK;
}

const char *reg_last_error(const reg_ctx *ctx) { return ctx ? ctx->err.c_str() : "null context"; }

reg_status reg_set_beta(reg_ctx *ctx, double beta) {
    CTX_OK(ctx);
    if (!(beta > 0) || !std::isfinite(beta)) return fail(ctx, REG_EINVAL, "beta must be positive and finite");
    ctx->beta = beta;
    ctx->P.beta = beta;
    return REG_OK;
}

reg_status reg_set_images(reg_ctx *ctx, const void *rho_T, const void *rho_R) {
    CTX_OK(ctx);
    NEED_DEV(ctx, rho_T);
    NEED_DEV(ctx, rho_R);
    const long N = ctx->N;
    if (ctx->P.prec) {
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(N, CV<double>(rho_T), V<double>(ctx->rhoT), ctx->stream)));
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(N, CV<double>(rho_R), V<double>(ctx->rhoR), ctx->stream)));
        STCHK(reduce<double>(ctx, ctx->rhoT, ctx->rhoR, N, 1, h3(ctx), 0));
    } else {
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<float>(N, CV<float>(rho_T), V<float>(ctx->rhoT), ctx->stream)));
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<float>(N, CV<float>(rho_R), V<float>(ctx->rhoR), ctx->stream)));
        STCHK(reduce<float>(ctx, ctx->rhoT, ctx->rhoR, N, 1, h3(ctx), 0));
    }
    STCHK(fetch(ctx, 1));
    ctx->normTR2 = ctx->hres[0];
    ctx->have_images = true;
    ctx->have_state = false;
    return REG_OK;
}

reg_status reg_interp(reg_ctx *ctx, const void *f, const void *D, void *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, f);
    NEED_DEV(ctx, D);
    NEED_DEV(ctx, out);
    if (f == out) return fail(ctx, REG_EINVAL, "out must not alias f");
    ctx->interps++;
    if (ctx->P.prec) {
        STCHK(measure_plan<double>(ctx, D));
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<double>(ctx->g, CV<double>(f), CV<double>(D), V<double>(out), ctx->stream, geom_of(ctx, D))));
    } else {
        STCHK(measure_plan<float>(ctx, D));
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<float>(ctx->g, CV<float>(f), CV<float>(D), V<float>(out), ctx->stream, geom_of(ctx, D))));
    }
    return REG_OK;
}

reg_status reg_backtrace(reg_ctx *ctx, const void *v, double sign, void *D) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, D);
    if (sign != 1.0 && sign != -1.0) return fail(ctx, REG_EINVAL, "sign must be +1 or -1");
    if (v == D) return fail(ctx, REG_EINVAL, "D must not alias v");
    return DISPATCH(ctx, backtrace_impl, ctx, v, sign, D);
}

reg_status reg_deriv(reg_ctx *ctx, int axis, const void *u, void *du) {
    CTX_OK(ctx);
    NEED_DEV(ctx, u);
    NEED_DEV(ctx, du);
    if (axis < 0 || axis > 2) return fail(ctx, REG_EINVAL, "axis must be 0, 1 or 2");
    const long N = ctx->N;
    if (ctx->P.prec) HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<double>(ctx->spec, axis, CV<double>(u), N, V<double>(du), N, 0, 1, ctx->stream)));
    else HIPCHK(ctx, KL(ctx, REG_K_DERIV, regk::spec_deriv<float>(ctx->spec, axis, CV<float>(u), N, V<float>(du), N, 0, 1, ctx->stream)));
    return REG_OK;
}

reg_status reg_grad(reg_ctx *ctx, const void *u, void *g) {
    CTX_OK(ctx);
    NEED_DEV(ctx, u);
    NEED_DEV(ctx, g);
    return DISPATCH(ctx, gradient_fields, ctx, u, 1, g);
}

reg_status reg_div(reg_ctx *ctx, const void *v, void *d) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, d);
    return DISPATCH(ctx, divergence, ctx, v, d);
}

reg_status reg_spectral(reg_ctx *ctx, int op, double scale, int ncomp, const void *v, void *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, out);
    if (op < 0 || op > 3) return fail(ctx, REG_EINVAL, "op must be 0..3");
    if (ncomp != 1 && ncomp != 3) return fail(ctx, REG_EINVAL, "ncomp must be 1 or 3");
    if (op == 3 && ncomp != 3) return fail(ctx, REG_EINVAL, "the Leray projection needs 3 components");
    if ((op == 0 || op == 1) && !(scale > 0)) return fail(ctx, REG_EINVAL, "scale must be positive");
    if (!std::isfinite(scale)) return fail(ctx, REG_EINVAL, "scale must be finite");
    return DISPATCH(ctx, spectral_impl, ctx, op, scale, ncomp, v, out);
}

reg_status reg_precond(reg_ctx *ctx, const void *r, void *z) {
    CTX_OK(ctx);
    NEED_DEV(ctx, r);
    NEED_DEV(ctx, z);
    return precond_impl(ctx, r, z);
}

reg_status reg_transport_forward(reg_ctx *ctx, const void *v, const void *rho0, void *rho1) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, rho0);
    NEED_DEV(ctx, rho1);
    return DISPATCH(ctx, transport_forward_impl, ctx, v, rho0, rho1);
}

reg_status reg_transport_adjoint(reg_ctx *ctx, const void *v, const void *lam1, void *lam0) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, lam1);
    NEED_DEV(ctx, lam0);
    return DISPATCH(ctx, transport_adjoint_impl, ctx, v, lam1, lam0);
}

reg_status reg_gradient(reg_ctx *ctx, const void *v, void *g, double *J, double *mismatch, double *gnorm) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, g);
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    ctx->have_state = false;
    return DISPATCH(ctx, gradient_impl, ctx, v, g, J, mismatch, gnorm, false);
}

reg_status reg_objective(reg_ctx *ctx, const void *v, double *J, double *mismatch) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    if (!J || !mismatch) return fail(ctx, REG_EINVAL, "J and mismatch are required");
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    return DISPATCH(ctx, trial_objective, ctx, v, J, mismatch);
}

reg_status reg_hessian_matvec(reg_ctx *ctx, const void *vt, void *Hvt) {
    CTX_OK(ctx);
    NEED_DEV(ctx, vt);
    NEED_DEV(ctx, Hvt);
    if (!ctx->have_state) return fail(ctx, REG_EINVAL, "reg_gradient must be called first");
    return DISPATCH(ctx, matvec_impl, ctx, vt, Hvt);
}

reg_status reg_solve(reg_ctx *ctx, void *v_inout, reg_report *rep) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v_inout);
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    reg_report local;
    reg_report *r = rep ? rep : &local;
    std::memset(r, 0, sizeof(*r));
    ctx->have_state = false;
    reg_status st = DISPATCH(ctx, solve_impl, ctx, v_inout, r);
    r->status = st;
    return st;
}

reg_status reg_deformation(reg_ctx *ctx, const void *v, void *u_or_null, double *detmin, double *detmax) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    if (u_or_null) NEED_DEV(ctx, u_or_null);
    if (!detmin || !detmax) return fail(ctx, REG_EINVAL, "detmin and detmax are required");
    return DISPATCH(ctx, deformation_impl, ctx, v, u_or_null, detmin, detmax);
}

reg_status reg_dot(reg_ctx *ctx, int ncomp, const void *a, const void *b, double *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, a);
    NEED_DEV(ctx, b);
    if (!out || ncomp < 1) return fail(ctx, REG_EINVAL, "bad arguments");
    reg_status st = reduce<double>(ctx, a, b, ncomp * ctx->N, 0, h3(ctx), 0);
    if (st != REG_OK) return st;
    STCHK(fetch(ctx, 1));
    *out = ctx->hres[0];
    return REG_OK;
}

reg_status reg_profile(reg_ctx *ctx, int enable) {
    CTX_OK(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    prof_resolve(ctx);
    for (int k = 0; k < REG_K_COUNT; k++) {
        if (enable) {
            ctx->prof_ms[k] = 0;
            ctx->prof_n[k] = 0;
        }
    }
    ctx->prof_on = enable != 0;
    return REG_OK;
}

reg_status reg_profile_read(reg_ctx *ctx, int kind, int64_t *launches, double *ms) {
    CTX_OK(ctx);
    if (kind < 0 || kind >= REG_K_COUNT || !launches || !ms) return fail(ctx, REG_EINVAL, "bad profile query");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    prof_resolve(ctx);
    *launches = ctx->prof_n[kind];
    *ms = ctx->prof_ms[kind];
    return REG_OK;
}

}  // extern "C"
