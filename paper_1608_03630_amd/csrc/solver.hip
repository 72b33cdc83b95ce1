// Gauss-Newton-Krylov driver of section III-A (reduced-space inexact Newton
// with truncated PCG, the spectral preconditioner, forcing sequence, Armijo
// backtracking and beta continuation) and the executor of its heavy
// operations: the reduced gradient (state, adjoint, eq. (4)), the objective
// (state) and the Gauss-Newton Hessian matvec (incremental state and
// incremental adjoint, eqs. (5a)-(5e) without the second-order terms).
//
// One executor serves a single problem (reg_gradient, reg_solve, ...) and a
// batch of independent problems of mixed sizes on one stream (reg_batch_*).
// Every problem's solver is an explicit state machine. The executor works in
// rounds: each active problem has queued light work (vector updates,
// preconditioner, inner products) and at most one heavy request; the round
// issues all heavy requests -- in a batch every semi-Lagrangian time step of
// all problems goes out as one persistent launch per LDS box class over a
// (problem, tile) work list -- then synchronises the stream once, and every
// problem reads its double-precision scalars and advances to its next
// request. In a batch the
// Hessian matvecs of a round are replayed from a captured HIP graph when the
// same set of problems repeats them. Per problem, the kernels and their
// arguments are those of the single-problem path, so a problem's result does
// not depend on the batch it runs in.
#include <algorithm>
#include <cstdio>
#include <functional>
#include <map>
#include <memory>
#include <mutex>

#include "ctx.hpp"

using namespace regc;

namespace {

enum class Op { NONE, GRADIENT, OBJECTIVE, MATVEC, FORWARD };

// A heavy operation of one problem.
struct Request {
    Op op = Op::NONE;
    const void *x = nullptr;    // v (GRADIENT, OBJECTIVE, FORWARD) or vt (MATVEC), velocity space
    void *y = nullptr;          // g (GRADIENT), Hvt (MATVEC), rho1 (FORWARD)
    const void *aux = nullptr;  // rho0 (FORWARD)
    bool reuse = false;         // GRADIENT: histB and Dt already hold the plan and state of x
    bool dot = false;           // MATVEC: <vt, Hvt> into result slot 0
    bool pre = false;           // MATVEC: x is a Krylov vector (complex field type), transformed in place
};

struct Item {
    reg_ctx *ctx;
    Request req;
};

int slots_of(const Request &r) {
    switch (r.op) {
    case Op::GRADIENT: return 4;
    case Op::OBJECTIVE: return 3;
    case Op::MATVEC: return r.dot ? 1 : 0;
    default: return 0;
    }
}

// ------------------------------------------------------------- autotuner
// Launch shape of the batched step kernel (workgroup count and XCD dealing)
// per (mode, box span, set of grid sizes), measured on first use and kept for
// the process.
struct TuneEntry {
    int blocks = 0;
    int chunked = 1;
    int t1 = regk::kTile1, t2 = regk::kTile2;  // tile shape t1 x t2 x 64
    double ms = 0;
};
std::mutex g_tune_mu;
std::map<std::string, TuneEntry> g_tune;

}  // namespace

// --------------------------------------------------------------- the batch
struct reg_batch {
    int npairs = 0;
    int prec = 0;
    int nt_max = 0;
    std::vector<reg_ctx *> ctx;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    regc::Profiler prof;
    // device tables of PairStep: region 0 for a round's eager gradients,
    // objectives and transports, region 1 for its eager matvecs, 2 + i for
    // cached graph i
    regk::PairStep *dev_tab = nullptr;
    regk::PairStep *host_tab = nullptr;  // pinned staging, same layout
    size_t region = 0;                   // entries per region
    static constexpr int kGraphs = 4;
    // launch configuration
    int fixed_blocks = 0;  // 0: autotune
    int fixed_chunked = 1;
    int fixed_t1 = 0, fixed_t2 = 0;  // 0: tile shape autotuned
    int use_graph = 1;
    struct GraphEntry {
        std::vector<int64_t> key;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        uint64_t used = 0;
    };
    GraphEntry graphs[kGraphs];
    std::vector<int64_t> last_key;
    uint64_t tick = 0;
    int64_t launches = 0, captures = 0, replays = 0;
    TuneEntry last[3];
    int last_variant[3] = {0, 0, 0};
    std::string err;
};

namespace {

// ---------------------------------------------------------------- program
// The GPU work of a round, built first (so that the batched step tables can
// be uploaded in one copy) and then run, eagerly or under stream capture.
struct Program {
    std::vector<std::function<reg_status()>> ops;
    std::vector<regk::PairStep> table;
};

reg_status bfail(reg_batch *b, reg_status st, const std::string &msg) {
    if (b) b->err = msg;
    return st;
}

int kind_of_mode(int mode) {
    return mode == regk::STEP_INTERP ? REG_K_INTERP : mode == regk::STEP_ADJOINT ? REG_K_ADJOINT : REG_K_INCSTATE;
}

// One batched step launch: mode, kernel variant, dynamic LDS, table; total
// counts unit tiles (regk::unit_tiles_of).
struct Launch {
    int mode = 0, variant = 0, n = 0, total = 0;
    size_t lds = 0;
    const regk::PairStep *dev = nullptr;
};

std::string tune_key(const Launch &L, const regk::PairStep *p, size_t esz) {
    std::vector<std::string> sizes;
    for (int i = 0; i < L.n; i++)
        sizes.push_back(std::to_string(p[i].g.n1) + "x" + std::to_string(p[i].g.n2) + "x" + std::to_string(p[i].g.n3));
    std::sort(sizes.begin(), sizes.end());
    // the dynamic LDS enters by occupancy class (16 KB steps), so that boxes
    // that drift with the velocity do not trigger new tuning
    std::string k = std::to_string(esz) + "/" + std::to_string(L.mode) + "/" + std::to_string(L.variant) + "/" +
                    std::to_string((L.lds + 16383) / 16384);
    for (auto &s : sizes) k += "/" + s;
    return k;
}

// Runs a batched step launch with the launch shape from the tuner (tuning it
// here, by timing every candidate on this very launch, when the shape is not
// known yet and the stream is not being captured; every candidate computes
// the same output from the same inputs).
// tile shapes t1 x t2 x 64 that a launch can take: the box of the variant
// fits, and every problem's grid is made of whole tiles
std::vector<std::pair<int, int>> tile_shapes(const Launch &L, const regk::PairStep *host) {
    std::vector<std::pair<int, int>> out;
    if (L.variant == 0) return {{regk::kTile1, regk::kTile2}};  // the generic kernel: default tiles
    for (int i = 0; i < regk::kBatchTileCount; i++) {
        const int t1 = regk::kBatchTiles[i][0], t2 = regk::kBatchTiles[i][1];
        if (!regk::batch_tile_ok(L.variant, t1, t2)) continue;
        bool ok = true;
        for (int p = 0; p < L.n && ok; p++) ok = host[p].g.n1 % t1 == 0 && host[p].g.n2 % t2 == 0;
        if (ok) out.push_back({t1, t2});
    }
    return out;
}

template <typename T>
reg_status batched_launch(reg_batch *b, const Launch &L, const regk::PairStep *host, bool capturing) {
    TuneEntry e;
    bool have = false;
    const std::string key = tune_key(L, host, sizeof(T));
    // work items of a shape: the launch's unit tiles / the unit tiles per tile
    auto units = [&](int t1, int t2) { return L.variant == 0 ? 1 : (t1 / regk::kUnit1) * (t2 / regk::kUnit2); };
    auto go = [&](int nb, int chunked, int t1, int t2) {
        const int ratio = units(t1, t2);
        return regk::launch_batched_step<T>(L.mode, L.variant, L.lds, L.dev, L.n, L.total / ratio,
                                            std::max(8, std::min(nb, L.total / ratio)), chunked, t1, t2, b->stream);
    };
    const auto shapes = tile_shapes(L, host);
    if (shapes.empty()) return bfail(b, REG_EINVAL, "no tile shape fits a batched launch");
    bool fixed_tile = false;
    for (const auto &sh : shapes)
        if (sh.first == b->fixed_t1 && sh.second == b->fixed_t2) fixed_tile = true;
    if (b->fixed_blocks > 0) {
        e.blocks = b->fixed_blocks;
        e.chunked = b->fixed_chunked;
        e.t1 = fixed_tile ? b->fixed_t1 : shapes[0].first;
        e.t2 = fixed_tile ? b->fixed_t2 : shapes[0].second;
        have = true;
    } else if (fixed_tile) {
        // a fixed tile with autotuned blocks: a key of its own
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key + "/t" + std::to_string(b->fixed_t1) + "x" + std::to_string(b->fixed_t2));
        if (it != g_tune.end()) {
            e = it->second;
            have = true;
        }
    } else {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(key);
        if (it != g_tune.end()) {
            e = it->second;
            have = true;
        }
    }
    if (!have && capturing) {  // no timing under capture: a safe default
        e.blocks = 1024;
        e.chunked = 1;
        e.t1 = fixed_tile ? b->fixed_t1 : shapes[0].first;
        e.t2 = fixed_tile ? b->fixed_t2 : shapes[0].second;
        have = true;
    }
    if (!have) {
        // tile shapes (or the fixed one) x workgroup counts (powers of two,
        // multiples of 768 for boxes that fit three workgroups per CU, and
        // all tiles) x XCD dealing, each timed on this very launch; every
        // candidate computes the same output from the same inputs
        std::vector<std::pair<int, int>> cand_shapes = shapes;
        if (fixed_tile) cand_shapes = {{b->fixed_t1, b->fixed_t2}};
        const std::vector<int> cand = {256, 512, 768, 1024, 1536, 2048, 3072, 4096, 1 << 30};
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
            hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess)
            return bfail(b, REG_EHIP, "hipEventCreate failed in the launch tuner");
        TuneEntry best;
        best.ms = 1e30;
        reg_status st = REG_OK;
        for (const auto &sh : cand_shapes) {
            const int items = L.total / units(sh.first, sh.second);
            for (int chunked = 1; chunked >= 0 && st == REG_OK; chunked--) {
                for (int c : cand) {
                    const int nb = std::max(8, std::min(c, items));
                    hipError_t he = go(nb, chunked, sh.first, sh.second);
                    if (he == hipSuccess) he = hipEventRecord(e0, b->stream);
                    if (he == hipSuccess) he = go(nb, chunked, sh.first, sh.second);
                    if (he == hipSuccess) he = hipEventRecord(e1, b->stream);
                    if (he == hipSuccess) he = hipEventSynchronize(e1);
                    float ms = 0;
                    if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                    if (he != hipSuccess) {
                        st = bfail(b, REG_EHIP, std::string("launch tuner: ") + hipGetErrorString(he));
                        break;
                    }
                    if (ms < best.ms) {
                        best.ms = ms;
                        best.blocks = nb;
                        best.chunked = chunked;
                        best.t1 = sh.first;
                        best.t2 = sh.second;
                    }
                    if (c >= items) break;
                }
            }
            if (st != REG_OK) break;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        if (st != REG_OK) return st;
        e = best;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[fixed_tile ? key + "/t" + std::to_string(b->fixed_t1) + "x" + std::to_string(b->fixed_t2) : key] = e;
    }
    hipError_t he = timed(b->prof, kind_of_mode(L.mode), [&]() { return go(e.blocks, e.chunked, e.t1, e.t2); });
    if (he != hipSuccess) return bfail(b, REG_EHIP, std::string("batched step launch: ") + hipGetErrorString(he));
    b->launches++;
    b->last[L.mode] = e;
    b->last_variant[L.mode] = L.variant;
    return REG_OK;
}

// Full Newton Hessian matvec of one context (eqs. (5a)-(5e) with both lam
// terms; single contexts only), from the plans, state history, grad rho^n,
// div v and its Heun factor of the last gradient and that gradient's adjoint
// levels (lamg):
// * incremental state with every level kept (histB, free between a gradient
//   and the next line search): the fused form q^{n+1} = q^n(X) - dt s^{n+1},
//   s = vt . grad rho, with rho~^n = q^n + dt/2 s^n;
// * incremental adjoint from lam~(1) = -rho~(1) with the source
//   s~ = div(lam vt): each step (eq. (7) expanded) is
//   lam~(X) gam + s~^k(X) dt/2 (1 + dt c) + dt/2 s~^{k-1};
// * b~ = sum_n w_n (lam~^n grad rho^n + lam^n grad rho~^n), then the
//   assembly of the Gauss-Newton matvec.
// Scratch: du (lam vt and grad rho~^n) and u0 (two source levels and s~(X)).
// b = sum_n w_n lam^n grad rho^n (trapezoid weights, eqs. (4), (5e)) from the
// kept levels of grad rho in one pass, or, with recompute_grad_rho, level by
// level: grad rho^n of the state history into the one kept level, then
// b += w_n lam^n grad rho^n (the same products and order of additions).
template <typename T>
reg_status b_sum(reg_ctx *ctx, const T *lam, T *b) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    if (!ctx->P.recompute_grad_rho) {
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_b_assemble<T>(N, nt, lam, CV<T>(ctx->grho), b, ctx->stream)));
        return REG_OK;
    }
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_fill<T>(3 * N, 0.0, b, ctx->stream)));
    for (int n = 0; n <= nt; n++) {
        const double w = (n == 0 || n == nt) ? 0.5 / nt : 1.0 / nt;
        STCHK(gradient_fields<T>(ctx, CV<T>(ctx->histA) + (long)n * N, 1, ctx->grho));
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_b_axpy<T>(N, w, lam + (long)n * N, CV<T>(ctx->grho), b,
                                                                 ctx->stream)));
    }
    return REG_OK;
}

template <typename T>
reg_status newton_matvec(reg_ctx *ctx, const Request &r) {
    const long N = ctx->N;
    const int nt = ctx->P.nt;
    const double dt = 1.0 / nt;
    hipStream_t st = ctx->stream;
    if (r.pre) STCHK(field_from_krylov<T>(ctx, r.x, ctx->vtf));
    else STCHK(spec_to_field<T>(ctx, r.x, ctx->vtf));
    const T *vt = CV<T>(ctx->vtf), *grho = CV<T>(ctx->grho), *lamg = CV<T>(ctx->lamg);
    T *rt = V<T>(ctx->histB), *lam = V<T>(ctx->lamh), *bt = V<T>(ctx->bvec), *w3 = V<T>(ctx->du);
    T *s_cur = V<T>(ctx->u0), *s_next = s_cur + N, *sX = s_cur + 2 * N;
    // incremental state: q^0 = -dt/2 s^0, q^{k+1} = q^k(X) - dt s^{k+1},
    // the last step rho~^nt = q^{nt-1}(X) - dt/2 s^nt
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_incstate_init<T>(ctx->g, vt, grho, rt, -0.5 * dt, st)));
    for (int k = 0; k < nt; k++) {
        const bool last = k == nt - 1;
        HIPCHK(ctx, KL(ctx, REG_K_INCSTATE, regk::launch_incstate_step<T>(
                                                ctx->g, rt + (long)k * N, CV<T>(ctx->Df), vt, grho + (long)(k + 1) * 3 * N,
                                                rt + (long)(k + 1) * N, last ? -0.5 * dt : -dt, 0, st,
                                                geom_of(ctx, ctx->Df))));
    }
    // rho~^k = q^k + dt/2 s^k (k = 1..nt-1); rho~^0 = 0
    for (int k = 1; k < nt; k++)
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_add_vdotgrad<T>(N, vt, grho + (long)k * 3 * N, rt + (long)k * N,
                                                                      0.5 * dt, st)));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_fill<T>(N, 0.0, rt, st)));
    // lam~(1) = -rho~(1)
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_scale<T>(N, -1.0, rt + (long)nt * N, lam + (long)nt * N, st)));
    // incremental adjoint with the source div(lam vt)
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_scale_vec<T>(N, lamg + (long)nt * N, vt, w3, st)));
    STCHK(divergence<T>(ctx, w3, s_cur));
    const T *gam = ctx->P.isochoric ? nullptr : CV<T>(ctx->gam);
    const T *cdiv = ctx->P.isochoric ? nullptr : CV<T>(ctx->c);
    for (int k = nt; k > 0; k--) {
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_scale_vec<T>(N, lamg + (long)(k - 1) * N, vt, w3, st)));
        STCHK(divergence<T>(ctx, w3, s_next));
        HIPCHK(ctx, KL(ctx, REG_K_ADJOINT, regk::launch_adjoint_step<T>(ctx->g, lam + (long)k * N, CV<T>(ctx->Da), gam,
                                                                        lam + (long)(k - 1) * N, st,
                                                                        geom_of(ctx, ctx->Da))));
        HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, s_cur, CV<T>(ctx->Da), sX, st,
                                                                 geom_of(ctx, ctx->Da))));
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_newton_source<T>(N, sX, s_next, cdiv, dt, lam + (long)(k - 1) * N,
                                                                        st)));
        std::swap(s_cur, s_next);
    }
    // b~ = sum_n w_n lam~^n grad rho^n + sum_n w_n lam^n grad rho~^n
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_b_assemble<T>(N, nt, lam, grho, bt, st)));
    for (int k = 0; k <= nt; k++) {
        const double w = (k == 0 || k == nt) ? 0.5 * dt : dt;
        STCHK(gradient_fields<T>(ctx, rt + (long)k * N, 1, w3));
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_b_axpy<T>(N, w, lamg + (long)k * N, w3, bt, st)));
    }
    if (r.pre) return curvature<T>(ctx, r.x, ctx->bvec, 0);
    return assemble<T>(ctx, r.x, ctx->bvec, r.y, r.dot ? 1 : 0, 0);
}

// Operands of one semi-Lagrangian step of one problem.
template <typename T>
struct StepArg {
    reg_ctx *ctx;
    const T *f;
    const T *D;
    T *out;
    const T *gam = nullptr;
    const T *vt = nullptr;
    const T *grad = nullptr;
    double cs = 0;
    int last = 0;
};

template <typename T>
struct Exec {
    reg_batch *b;           // nullptr: single problems, no batched launches, no graphs
    hipStream_t stream;
    bool capturing = false;

    Exec(reg_batch *b_, hipStream_t s) : b(b_), stream(s) {}

    // queues one time step of every problem in args: a single batched launch
    // for the problems the canonical tile kernel takes, the single-problem
    // launchers for the rest
    void sl_step(Program &P, int mode, const std::vector<StepArg<T>> &args, const regk::PairStep *dev_region) {
        // Problems are grouped by LDS box class: canonical boxes of floor span
        // 1, 2 or 4 (classes 0..2) and the generic box (class 3). Each class
        // takes one batched launch over its (problem, tile) work list, so that
        // a problem with small steps keeps the small box (and four workgroups
        // per CU) whatever the other problems need.
        std::vector<regk::PairStep> items[4];
        int total[4] = {0, 0, 0, 0};
        size_t lds[4] = {0, 0, 0, 0};
        for (const auto &a : args) {
            const regk::TileGeom *tg = geom_of(a.ctx, a.D);
            if (b && tg) {
                regk::PairStep ps{};
                ps.g = a.ctx->g;
                ps.tg = *tg;
                ps.f = a.f;
                ps.D = a.D;
                ps.gam = a.gam;
                ps.grad = a.grad;
                ps.vt = a.vt;
                ps.out = a.out;
                ps.cs = a.cs;
                ps.last = a.last;
                ps.canon = regk::canonical(a.ctx->g, *tg, sizeof(T));
                const int span = regk::batch_span(*tg);
                const int cls = !ps.canon ? 3 : span <= 1 ? 0 : span <= 2 ? 1 : 2;
                // canonical classes count unit tiles (any batch tile shape
                // follows), the generic class the default tiles of its
                // possibly ragged grids
                ps.tile0 = total[cls];
                total[cls] += cls == 3 ? regk::tiles_of(a.ctx->g) : regk::unit_tiles_of(a.ctx->g);
                lds[cls] = std::max(lds[cls], sizeof(T) * (size_t)tg->B[0] * tg->B[1] * tg->B[2]);
                items[cls].push_back(ps);
                continue;
            }
            // no tile geometry (a box beyond the LDS) or a single problem: the
            // single-problem launchers
            const StepArg<T> c = a;
            P.ops.push_back([c, mode, tg]() -> reg_status {
                reg_ctx *ctx = c.ctx;
                if (mode == regk::STEP_INTERP)
                    HIPCHK(ctx, KL(ctx, REG_K_INTERP, regk::launch_interp<T>(ctx->g, c.f, c.D, c.out, ctx->stream, tg)));
                else if (mode == regk::STEP_ADJOINT)
                    HIPCHK(ctx, KL(ctx, REG_K_ADJOINT, regk::launch_adjoint_step<T>(ctx->g, c.f, c.D, c.gam, c.out, ctx->stream, tg)));
                else
                    HIPCHK(ctx, KL(ctx, REG_K_INCSTATE, regk::launch_incstate_step<T>(ctx->g, c.f, c.D, c.vt, c.grad, c.out, c.cs,
                                                                                      c.last, ctx->stream, tg)));
                return REG_OK;
            });
        }
        static const int kVariant[4] = {1, 2, 4, 0};
        for (int cls = 0; cls < 4; cls++) {
            if (items[cls].empty()) continue;
            Launch L;
            L.mode = mode;
            L.n = (int)items[cls].size();
            L.total = total[cls];
            L.variant = kVariant[cls];
            L.lds = cls == 3 ? lds[cls] : 0;
            const size_t off = P.table.size();
            P.table.insert(P.table.end(), items[cls].begin(), items[cls].end());
            L.dev = dev_region + off;
            P.ops.push_back([this, L, off, &P]() -> reg_status {
                return batched_launch<T>(b, L, P.table.data() + off, capturing);
            });
        }
    }

    // ---------------------------------------------------------------- plans
    // Phase A of a round: departure points and their floor bounds for every
    // request that needs new plans, one synchronisation for all.
    reg_status plans(std::vector<Item> &items) {
        bool any = false;
        for (auto &it : items) {
            reg_ctx *ctx = it.ctx;
            const long N3 = 3 * ctx->N;
            const Request &r = it.req;
            if (r.op == Op::GRADIENT) {
                if (r.x != ctx->vhat)
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(sv_len(ctx), CV<double>(r.x), V<double>(ctx->vhat), ctx->stream)));
                STCHK(spec_to_field<T>(ctx, ctx->vhat, ctx->vf));
                if (r.reuse) {
                    std::swap(ctx->histA, ctx->histB);
                    std::swap(ctx->Df, ctx->Dt);
                    ctx->epoch++;
                } else {
                    STCHK(plan_enqueue<T>(ctx, ctx->vf, +1.0, ctx->Df, ctx->dpart, kSlotPlanA));
                }
                STCHK(plan_enqueue<T>(ctx, ctx->vf, -1.0, ctx->Da, ctx->dpart2, kSlotPlanB));
            } else if (r.op == Op::OBJECTIVE || r.op == Op::FORWARD) {
                if (r.op == Op::OBJECTIVE) STCHK(spec_to_field<T>(ctx, r.x, ctx->vf));  // spectral velocity
                else HIPCHK(ctx, KL(ctx, REG_K_VECTOR, to_field<T>(ctx, r.x, ctx->vf, N3)));  // physical velocity
                STCHK(plan_enqueue<T>(ctx, ctx->vf, +1.0, ctx->Dt, ctx->dpart, kSlotPlanA));
            } else {
                continue;
            }
            HIPCHK(ctx, hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * (kSlotPlanB + 6), hipMemcpyDeviceToHost,
                                       ctx->stream));
            any = true;
        }
        if (!any) return REG_OK;
        HIPCHK(items[0].ctx, hipStreamSynchronize(stream));
        for (auto &it : items) {
            reg_ctx *ctx = it.ctx;
            const Request &r = it.req;
            if (r.op == Op::GRADIENT) {
                if (!r.reuse) plan_finish(ctx, ctx->Df, kSlotPlanA);
                plan_finish(ctx, ctx->Da, kSlotPlanB);
            } else if (r.op == Op::OBJECTIVE || r.op == Op::FORWARD) {
                plan_finish(ctx, ctx->Dt, kSlotPlanA);
            }
        }
        return REG_OK;
    }

    // -------------------------------------------------------------- program
    // Phase B: the transport solves and everything after them, for the given
    // items (plans already in place).
    void build(Program &P, const std::vector<Item> &items, const regk::PairStep *dev_region) {
        int ntmax = 0;
        for (const auto &it : items) ntmax = std::max(ntmax, it.ctx->P.nt);
        // set-up of the forward-in-time solves
        for (const auto &it : items) {
            reg_ctx *ctx = it.ctx;
            const Request r = it.req;
            const long N = ctx->N;
            if (r.op == Op::GRADIENT && !r.reuse) {
                P.ops.push_back([ctx]() -> reg_status {
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(ctx->N, CV<T>(ctx->rhoT), V<T>(ctx->histA), ctx->stream)));
                    return REG_OK;
                });
            } else if (r.op == Op::OBJECTIVE) {
                P.ops.push_back([ctx]() -> reg_status {
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(ctx->N, CV<T>(ctx->rhoT), V<T>(ctx->histB), ctx->stream)));
                    return REG_OK;
                });
            } else if (r.op == Op::MATVEC) {
                // incremental state through q^n = rho~^n - dt/2 vt.grad rho^n
                const double dt = 1.0 / ctx->P.nt;
                P.ops.push_back([ctx, r, N, dt]() -> reg_status {
                    (void)N;
                    if (r.pre) STCHK(field_from_krylov<T>(ctx, r.x, ctx->vtf));
                    else STCHK(spec_to_field<T>(ctx, r.x, ctx->vtf));
                    if (ctx->P.recompute_grad_rho) STCHK(gradient_fields<T>(ctx, ctx->histA, 1, ctx->grho));
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_incstate_init<T>(ctx->g, CV<T>(ctx->vtf), V<T>(ctx->grho),
                                                                                    V<T>(ctx->lam[1]), -0.5 * dt, ctx->stream)));
                    return REG_OK;
                });
            }
        }
        // forward-in-time steps: state histories (one launch per step) and
        // incremental states (one launch per step)
        for (int k = 0; k < ntmax; k++) {
            std::vector<StepArg<T>> fw, inc;
            for (const auto &it : items) {
                reg_ctx *ctx = it.ctx;
                const Request &r = it.req;
                const int nt = ctx->P.nt;
                const long N = ctx->N;
                if (k >= nt) continue;
                if (r.op == Op::GRADIENT && !r.reuse) {
                    fw.push_back({ctx, CV<T>(ctx->histA) + k * N, CV<T>(ctx->Df), V<T>(ctx->histA) + (k + 1) * N});
                } else if (r.op == Op::OBJECTIVE) {
                    fw.push_back({ctx, CV<T>(ctx->histB) + k * N, CV<T>(ctx->Dt), V<T>(ctx->histB) + (k + 1) * N});
                } else if (r.op == Op::FORWARD) {
                    // ping-pong between two slices of the scratch history, last step into rho1
                    const T *src = k == 0 ? CV<T>(r.aux) : CV<T>(ctx->histB) + (long)((k - 1) & 1) * N;
                    T *dst = (k == nt - 1) ? V<T>(r.y) : V<T>(ctx->histB) + (long)(k & 1) * N;
                    fw.push_back({ctx, src, CV<T>(ctx->Dt), dst});
                } else if (r.op == Op::MATVEC) {
                    const int last = (k == nt - 1);
                    const double dt = 1.0 / nt;
                    const int cur = (k & 1) ? 0 : 1;  // lam[1] holds q^0
                    StepArg<T> a{ctx, CV<T>(ctx->lam[cur]), CV<T>(ctx->Df),
                                 last ? V<T>(ctx->lamh) + (long)nt * N : V<T>(ctx->lam[1 - cur])};
                    a.vt = CV<T>(ctx->vtf);
                    a.grad = CV<T>(ctx->grho) + (ctx->P.recompute_grad_rho ? 0 : (long)(k + 1) * 3 * N);
                    a.cs = last ? -0.5 * dt : -dt;
                    a.last = last;
                    inc.push_back(a);
                }
            }
            sl_step(P, regk::STEP_INTERP, fw, dev_region);
            // grad rho^{k+1} of the contexts that recompute it, just before the step reads it
            for (const auto &a : inc) {
                reg_ctx *ctx = a.ctx;
                if (!ctx->P.recompute_grad_rho) continue;
                P.ops.push_back([ctx, k]() -> reg_status {
                    return gradient_fields<T>(ctx, CV<T>(ctx->histA) + (long)(k + 1) * ctx->N, 1, ctx->grho);
                });
            }
            sl_step(P, regk::STEP_INCSTATE, inc, dev_region);
        }
        // gradient: grad rho^n, div v and its Heun factor, adjoint final value
        std::vector<StepArg<T>> cint;
        for (const auto &it : items) {
            if (it.req.op != Op::GRADIENT) continue;
            reg_ctx *ctx = it.ctx;
            P.ops.push_back([ctx]() -> reg_status {
                // (recomputed level by level in the b sum otherwise)
                if (!ctx->P.recompute_grad_rho) STCHK(gradient_fields<T>(ctx, ctx->histA, ctx->P.nt + 1, ctx->grho));
                if (!ctx->P.isochoric) STCHK(divergence<T>(ctx, ctx->vf, ctx->c));
                return REG_OK;
            });
            if (!ctx->P.isochoric) cint.push_back({ctx, CV<T>(ctx->c), CV<T>(ctx->Da), V<T>(ctx->cX)});
        }
        sl_step(P, regk::STEP_INTERP, cint, dev_region);
        for (const auto &it : items) {
            if (it.req.op != Op::GRADIENT) continue;
            reg_ctx *ctx = it.ctx;
            P.ops.push_back([ctx]() -> reg_status {
                const long N = ctx->N;
                const int nt = ctx->P.nt;
                if (!ctx->P.isochoric)
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_gamma<T>(N, CV<T>(ctx->c), CV<T>(ctx->cX), V<T>(ctx->gam),
                                                                            1.0 / nt, ctx->stream)));
                // lam(1) = rho_R - rho(1)
                HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_adjoint_init<T>(N, CV<T>(ctx->rhoR), CV<T>(ctx->histA) + (long)nt * N,
                                                                               V<T>(ctx->lamh) + (long)nt * N, ctx->stream)));
                return REG_OK;
            });
        }
        // backward sweeps (adjoint and incremental adjoint, one launch per step)
        for (int s = 0; s < ntmax; s++) {
            std::vector<StepArg<T>> adj;
            for (const auto &it : items) {
                if (it.req.op != Op::GRADIENT && it.req.op != Op::MATVEC) continue;
                reg_ctx *ctx = it.ctx;
                const int nt = ctx->P.nt;
                if (s >= nt) continue;
                const int k = nt - 1 - s;
                const long N = ctx->N;
                StepArg<T> a{ctx, CV<T>(ctx->lamh) + (long)(k + 1) * N, CV<T>(ctx->Da), V<T>(ctx->lamh) + (long)k * N};
                a.gam = ctx->P.isochoric ? nullptr : CV<T>(ctx->gam);
                adj.push_back(a);
            }
            sl_step(P, regk::STEP_ADJOINT, adj, dev_region);
        }
        // b = sum_n w_n lam^n grad rho^n, assembly and scalars
        for (const auto &it : items) {
            reg_ctx *ctx = it.ctx;
            const Request r = it.req;
            P.ops.push_back([ctx, r]() -> reg_status {
                const long N = ctx->N;
                const int nt = ctx->P.nt;
                if (r.op == Op::GRADIENT || r.op == Op::MATVEC) STCHK(b_sum<T>(ctx, CV<T>(ctx->lamh), V<T>(ctx->bvec)));
                // the full Newton matvecs at this velocity need its adjoint history
                if (r.op == Op::GRADIENT && ctx->P.hessian)
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>((long)(nt + 1) * N, CV<T>(ctx->lamh),
                                                                           V<T>(ctx->lamg), ctx->stream)));
                if (r.op == Op::GRADIENT) {
                    // g^ = beta |k|^4 v^ + P FFT(b); J and |g|^2 by Parseval
                    STCHK(biharm_partials(ctx, ctx->vhat));
                    STCHK(objective_slots<T>(ctx, ctx->histA, ctx->vhat, true));
                    STCHK(assemble<T>(ctx, ctx->vhat, ctx->bvec, r.y, 2, 3));
                } else if (r.op == Op::OBJECTIVE) {
                    STCHK(objective_slots<T>(ctx, ctx->histB, r.x, false));
                } else if (r.op == Op::MATVEC) {
                    if (r.pre) STCHK(curvature<T>(ctx, r.x, ctx->bvec, 0));
                    else STCHK(assemble<T>(ctx, r.x, ctx->bvec, r.y, r.dot ? 1 : 0, 0));
                }
                return REG_OK;
            });
        }
    }

    // Interpolations and the algorithmic bytes of the item's transport steps
    // and pointwise field passes, in fields per point: a state step reads D
    // and the gathered field and writes one (5), an adjoint step also reads
    // its Heun factor (6; 5 when isochoric), an incremental-state step reads
    // vt and grad rho^n as well (11), the b assembly reads lam^n and
    // grad rho^n at every level and writes b. Plans, derivatives, transforms
    // and velocity-space passes count where they are launched.
    void count(const Item &it) {
        reg_ctx *ctx = it.ctx;
        const int nt = ctx->P.nt;
        const double adj = ctx->P.isochoric ? 5 : 6;
        // b sum: one pass over the kept levels, or (recomputed grad rho) a
        // zero fill and an update of b per level
        const double bsum = ctx->P.recompute_grad_rho ? 3 + 10.0 * (nt + 1) : 4.0 * (nt + 1) + 3;
        switch (it.req.op) {
        case Op::GRADIENT:
            ctx->interps += (it.req.reuse ? 0 : nt) + (ctx->P.isochoric ? 0 : 1) + nt;
            alg_fields(ctx, (it.req.reuse ? 0 : 2 + 5.0 * nt) + (ctx->P.isochoric ? 0 : 5 + 3) + 3 + adj * nt + bsum +
                                (ctx->P.hessian ? 2.0 * (nt + 1) : 0));
            break;
        case Op::OBJECTIVE:
            ctx->interps += nt;
            alg_fields(ctx, 2 + 5.0 * nt);
            break;
        case Op::FORWARD:
            ctx->interps += nt;
            alg_fields(ctx, 5.0 * nt);
            break;
        case Op::MATVEC:
            ctx->interps += (ctx->P.hessian ? 3 : 2) * nt;
            alg_fields(ctx, 7 + 11.0 * nt + adj * nt + bsum);
            // full Newton: rho~ from q, lam vt, the interpolated source and
            // its Heun update, and the lam grad rho~ part of b~
            if (ctx->P.hessian)
                alg_fields(ctx, 8.0 * (nt - 1) + 3 + 7.0 * (nt + 1) + 5.0 * nt + (adj - 1) * nt + 10.0 * (nt + 1));
            break;
        default: break;
        }
    }

    reg_status run_ops(Program &P) {
        for (auto &op : P.ops) STCHK(op());
        return REG_OK;
    }

    reg_status upload(Program &P, size_t region_index) {
        if (!b || P.table.empty()) return REG_OK;
        if (P.table.size() > b->region) return bfail(b, REG_EINVAL, "batched step table overflow");
        regk::PairStep *h = b->host_tab + region_index * b->region;
        std::copy(P.table.begin(), P.table.end(), h);
        hipError_t e = hipMemcpyAsync(b->dev_tab + region_index * b->region, h, sizeof(regk::PairStep) * P.table.size(),
                                      hipMemcpyHostToDevice, stream);
        if (e != hipSuccess) return bfail(b, REG_EHIP, std::string("table upload: ") + hipGetErrorString(e));
        return REG_OK;
    }

    // Matvec items through a captured graph: replayed when the same problems
    // (same plans, operands and beta) were captured before; captured when the
    // previous matvec round had the same key; otherwise run eagerly.
    reg_status matvec_graph(std::vector<Item> &mv) {
        std::vector<int64_t> key;
        for (const auto &it : mv) {
            key.push_back((int64_t)(intptr_t)it.ctx);
            key.push_back(it.ctx->epoch);
            key.push_back((int64_t)(intptr_t)it.req.x);
            key.push_back((int64_t)(intptr_t)it.req.y);
            key.push_back(it.req.dot);
            key.push_back(it.req.pre);
            int64_t bb;
            std::memcpy(&bb, &it.ctx->beta, sizeof(bb));
            key.push_back(bb);
        }
        b->tick++;
        for (auto &g : b->graphs) {
            if (g.exec && g.key == key) {
                g.used = b->tick;
                hipError_t e = timed(b->prof, REG_K_GRAPH, [&]() { return hipGraphLaunch(g.exec, stream); });
                if (e != hipSuccess) return bfail(b, REG_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
                b->replays++;
                b->last_key = key;
                return REG_OK;
            }
        }
        const bool capture = (key == b->last_key);
        b->last_key = key;
        int slot = 0;
        if (capture) {
            for (int i = 1; i < reg_batch::kGraphs; i++)
                if (b->graphs[i].used < b->graphs[slot].used) slot = i;
            auto &g = b->graphs[slot];
            if (g.exec) (void)hipGraphExecDestroy(g.exec);
            if (g.graph) (void)hipGraphDestroy(g.graph);
            g = reg_batch::GraphEntry{};
        }
        const size_t region_index = capture ? 2 + slot : 1;
        Program P;
        build(P, mv, b->dev_tab + region_index * b->region);
        STCHK(upload(P, region_index));
        if (!capture) return run_ops(P);
        // capture without event timing
        std::vector<bool> prof_was;
        for (auto &it : mv) {
            prof_was.push_back(it.ctx->prof.on);
            it.ctx->prof.on = false;
        }
        const bool bprof = b->prof.on;
        b->prof.on = false;
        capturing = true;
        hipError_t e = hipStreamBeginCapture(stream, hipStreamCaptureModeRelaxed);
        reg_status st = e == hipSuccess ? run_ops(P) : bfail(b, REG_EHIP, std::string("hipStreamBeginCapture: ") + hipGetErrorString(e));
        hipGraph_t graph = nullptr;
        if (e == hipSuccess) {
            hipError_t e2 = hipStreamEndCapture(stream, &graph);
            if (st == REG_OK && e2 != hipSuccess) st = bfail(b, REG_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
        }
        capturing = false;
        for (size_t i = 0; i < mv.size(); i++) mv[i].ctx->prof.on = prof_was[i];
        b->prof.on = bprof;
        if (st != REG_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return st;
        }
        hipGraphExec_t exec = nullptr;
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return bfail(b, REG_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
        }
        auto &g = b->graphs[slot];
        g.key = key;
        g.graph = graph;
        g.exec = exec;
        g.used = b->tick;
        b->captures++;
        e = timed(b->prof, REG_K_GRAPH, [&]() { return hipGraphLaunch(exec, stream); });
        if (e != hipSuccess) return bfail(b, REG_EHIP, std::string("hipGraphLaunch: ") + hipGetErrorString(e));
        return REG_OK;
    }

    // One round of heavy requests; scalars are copied to each problem's pinned
    // buffer and become valid after the caller synchronises the stream.
    reg_status round(std::vector<Item> &items) {
        if (items.empty()) return REG_OK;
        STCHK(plans(items));
        std::vector<Item> eager, mv;
        for (auto &it : items) {
            count(it);
            if (it.req.op == Op::MATVEC && it.ctx->P.hessian) STCHK(newton_matvec<T>(it.ctx, it.req));
            else if (b && b->use_graph && it.req.op == Op::MATVEC) mv.push_back(it);
            else eager.push_back(it);
        }
        if (!eager.empty()) {
            Program P;
            build(P, eager, b ? b->dev_tab : nullptr);
            STCHK(upload(P, 0));
            STCHK(run_ops(P));
        }
        if (!mv.empty()) STCHK(matvec_graph(mv));
        for (auto &it : items) {
            const int ns = slots_of(it.req);
            if (ns > 0)
                HIPCHK(it.ctx, hipMemcpyAsync(it.ctx->hres, it.ctx->dres, sizeof(double) * ns, hipMemcpyDeviceToHost, stream));
        }
        return REG_OK;
    }
};

// ------------------------------------------------------------ the solver
enum State {
    S_START,
    S_LEVEL,
    S_LEVEL_GRAD,
    S_NEWTON,
    S_PCG_START,
    S_MATVEC_DONE,
    S_RR_DONE,
    S_ARMIJO,
    S_ARMIJO_D,
    S_FALLBACK_D,
    S_LS_TRY,
    S_LS_DONE,
    S_NEWTON_GRAD,
    S_LEVEL_END,
    S_FINISH,
    S_DONE
};

// The Gauss-Newton-Krylov iteration of one problem as a state machine. Each
// call of advance() runs host logic and queues light work until the problem
// needs a heavy operation (req) or scalars of its queued work (wait).
struct Solver {
    reg_ctx *ctx = nullptr;
    void *v = nullptr;
    reg_report *rep = nullptr;
    int st = S_START;
    Request req;
    bool wait = false;
    reg_status status = REG_OK;
    double beta = 0, beta_final = 0, factor = 0.1;
    double J = 0, mis = 0, gnorm = 0, g0 = 0, eta = 0, rz = 0, d = 0, alpha = 1;
    int k = 0, it = 0, i = 0, iters = 0, l = 0, trials = 0;
    bool changed = false;  // an accepted step or the projection moved v
    bool start_hat = false;  // vhat already holds the first iterate (grid continuation)
    double beta_start = 0;   // > 0: the first continuation level (grid continuation resumes there)
    double gref_start = 0;   // > 0: that level's gradient reference, measured on the coarser grid
    bool first_level = true;
    clk::time_point t0;
    long interps0 = 0;
    double alg0 = 0;

    bool done() const { return st == S_DONE; }

    // reference of the gradient stopping test: the level's first gradient
    // norm, or the caller's absolute reference
    double gref() const { return ctx->P.gnorm_ref > 0 ? ctx->P.gnorm_ref : g0; }
    // the level's tolerance: gtol_level above beta_final when given
    double level_tol() const {
        return (ctx->P.gtol_level > 0 && beta > beta_final * (1 + 1e-12)) ? ctx->P.gtol_level : ctx->P.gtol;
    }

    void queue_fetch(int nslots) {
        (void)hipMemcpyAsync(ctx->hres, ctx->dres, sizeof(double) * nslots, hipMemcpyDeviceToHost, ctx->stream);
        wait = true;
    }

    void finish(reg_status s) {
        status = s;
        st = S_FINISH;
    }

    reg_status read_gradient() {
        scalars_to_J(ctx, &J, &mis);
        gnorm = std::sqrt(ctx->hres[3]);
        rep->gradients++;
        if (!std::isfinite(ctx->hres[1]) || !std::isfinite(ctx->hres[2]) || !std::isfinite(ctx->hres[3]))
            return fail(ctx, REG_ENONFINITE, "non-finite objective or gradient");
        return REG_OK;
    }

    template <typename T>
    reg_status advance() {
        const reg_params &P = ctx->P;
        const long NV = sv_len(ctx);
        req = Request{};
        wait = false;
        for (;;) {
            switch (st) {
            case S_START: {
                t0 = clk::now();
                interps0 = ctx->interps;
                alg0 = ctx->alg_bytes;
                // the iterate lives on the half spectrum until the solve ends
                if (!start_hat) STCHK(to_spec(ctx, v, ctx->vhat));
                if (P.isochoric) STCHK(leray_hat(ctx, ctx->vhat));
                changed = P.isochoric != 0 || start_hat;
                beta_final = P.beta_final > 0 ? P.beta_final : P.beta;
                factor = (P.beta_factor > 0 && P.beta_factor < 1) ? P.beta_factor : 0.1;
                beta = beta_start > 0 ? beta_start : P.beta;
                it = 0;
                st = S_LEVEL;
                break;
            }
            case S_LEVEL:
                ctx->beta = beta;
                req = Request{Op::GRADIENT, ctx->vhat, ctx->ghat, nullptr, false, false};
                st = S_LEVEL_GRAD;
                return REG_OK;
            case S_LEVEL_GRAD: {
                reg_status s = read_gradient();
                if (s != REG_OK) {
                    finish(s);
                    break;
                }
                g0 = (first_level && gref_start > 0) ? gref_start : gnorm;
                first_level = false;
                rep->stop_reason = 2;
                k = 0;
                st = S_NEWTON;
                break;
            }
            case S_NEWTON: {
                if (k >= P.max_newton) {
                    st = S_LEVEL_END;
                    break;
                }
                if (gnorm <= level_tol() * gref()) {
                    rep->stop_reason = 0;
                    st = S_LEVEL_END;
                    break;
                }
                if (P.mismatch_tol > 0 && mis <= P.mismatch_tol) {
                    rep->stop_reason = 1;
                    st = S_LEVEL_END;
                    break;
                }
                // forcing relative to the same reference as the stopping test
                const double ratio = gref() > 0 ? gnorm / gref() : 0.0;
                eta = P.forcing == 1 ? std::sqrt(ratio) : ratio;
                if (eta > 0.5) eta = 0.5;
                // truncated PCG on H s = -g from s = 0
                STCHK(pcg_start<T>(ctx, 0));
                queue_fetch(1);
                st = S_PCG_START;
                return REG_OK;
            }
            case S_PCG_START:
                rz = ctx->hres[0];
                i = 0;
                iters = 0;
                // the matvec reads p in place; only the curvature <p, H p> comes back
                req = Request{Op::MATVEC, ctx->phat, nullptr, nullptr, false, true, true};
                st = S_MATVEC_DONE;
                return REG_OK;
            case S_MATVEC_DONE: {
                const double kappa = ctx->hres[0];
                rep->matvecs++;
                iters = i + 1;
                if (!std::isfinite(kappa)) {
                    finish(fail(ctx, REG_ENONFINITE, "non-finite curvature in PCG"));
                    break;
                }
                if (kappa <= 0) {  // negative curvature: stop (steepest descent at the first iteration)
                    rep->negative_curvature++;
                    // (p = M r at the first iteration)
                    if (i == 0) HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(NV, CV<T>(ctx->phat), V<T>(ctx->shat), ctx->stream)));
                    st = S_ARMIJO;
                    break;
                }
                const double a = rz / kappa;
                // one pass: the update, z = M r for the next direction and
                // both inner products, so that one synchronisation serves the
                // forcing test and the next direction (z unused when the test
                // ends the iteration)
                STCHK(pcg_step<T>(ctx, a, 0, 4));
                queue_fetch(5);
                st = S_RR_DONE;
                return REG_OK;
            }
            case S_RR_DONE: {
                const double rr = ctx->hres[0], rz1 = ctx->hres[4];
                if (std::sqrt(rr) <= eta * gnorm) {
                    st = S_ARMIJO;
                    break;
                }
                i++;
                if (i >= P.max_pcg) {
                    st = S_ARMIJO;
                    break;
                }
                STCHK(pcg_direction<T>(ctx, rz1 / rz));
                rz = rz1;
                req = Request{Op::MATVEC, ctx->phat, nullptr, nullptr, false, true, true};
                st = S_MATVEC_DONE;
                return REG_OK;
            }
            case S_ARMIJO:
                STCHK(krylov_dot<T>(ctx, ctx->ghat, ctx->shat, 0));
                queue_fetch(1);
                st = S_ARMIJO_D;
                return REG_OK;
            case S_ARMIJO_D:
                d = ctx->hres[0];
                if (!(d < 0)) {
                    // not a descent direction (a truncated or indefinite
                    // solve, or round-off in the stored PCG vectors): take
                    // the preconditioned steepest descent step -M g, with
                    // d = <g, -M g> = -<r, M r> for r = -g
                    STCHK(pcg_start<T>(ctx, 0));
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<T>(NV, CV<T>(ctx->phat), V<T>(ctx->shat), ctx->stream)));
                    queue_fetch(1);
                    st = S_FALLBACK_D;
                    return REG_OK;
                }
                alpha = 1.0;
                l = 0;
                trials = 0;
                st = S_LS_TRY;
                break;
            case S_FALLBACK_D:
                d = -ctx->hres[0];
                rep->descent_fallbacks++;
                alpha = 1.0;
                l = 0;
                trials = 0;
                st = S_LS_TRY;
                break;
            case S_LS_TRY:
                if (l >= P.max_ls) {
                    finish(fail(ctx, REG_ELINESEARCH, "Armijo line search found no acceptable step"));
                    break;
                }
                trials++;
                STCHK(krylov_axpy<T>(ctx, ctx->vhat, alpha, ctx->shat, ctx->vthat));
                req = Request{Op::OBJECTIVE, ctx->vthat, nullptr, nullptr, false, false};
                st = S_LS_DONE;
                return REG_OK;
            case S_LS_DONE: {
                double Jt = 0, mist = 0;
                scalars_to_J(ctx, &Jt, &mist);
                rep->objectives++;
                if (!std::isfinite(Jt)) {
                    finish(fail(ctx, REG_ENONFINITE, "non-finite objective"));
                    break;
                }
                if (Jt <= J + P.armijo_c1 * alpha * d) {
                    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_copy<double>(NV, CV<double>(ctx->vthat), V<double>(ctx->vhat), ctx->stream)));
                    changed = true;
                    req = Request{Op::GRADIENT, ctx->vhat, ctx->ghat, nullptr, true, false};
                    st = S_NEWTON_GRAD;
                    return REG_OK;
                }
                alpha *= 0.5;
                l++;
                st = S_LS_TRY;
                break;
            }
            case S_NEWTON_GRAD: {
                reg_status s = read_gradient();
                if (s != REG_OK) {
                    finish(s);
                    break;
                }
                if (it < REG_MAXIT) {
                    rep->J[it] = J;
                    rep->mismatch[it] = mis;
                    rep->grel[it] = g0 > 0 ? gnorm / g0 : 0;
                    rep->alpha[it] = alpha;
                    rep->beta[it] = beta;
                    rep->pcg_iters[it] = iters;
                    rep->ls_trials[it] = trials;
                }
                if (ctx->log_fn) {
                    char line[512];
                    std::snprintf(line, sizeof(line),
                                  "{\"n\": [%d, %d, %d], \"step\": %d, \"beta\": %.6e, \"J\": %.17g, "
                                  "\"mismatch\": %.17g, \"grel\": %.17g, \"alpha\": %.17g, \"pcg\": %d, \"ls\": %d, "
                                  "\"matvecs\": %d, \"seconds\": %.6f}",
                                  ctx->P.n[0], ctx->P.n[1], ctx->P.n[2], it, beta, J, mis, g0 > 0 ? gnorm / g0 : 0.0,
                                  alpha, iters, trials, rep->matvecs, secs(t0));
                    ctx->log_fn(line, ctx->log_user);
                }
                it++;
                rep->stop_reason = 2;
                k++;
                st = S_NEWTON;
                break;
            }
            case S_LEVEL_END:
                if (rep->stop_reason == 2) {
                    if (gnorm <= level_tol() * gref()) rep->stop_reason = 0;
                    if (P.mismatch_tol > 0 && mis <= P.mismatch_tol) rep->stop_reason = 1;
                }
                if (rep->stop_reason == 1 || beta <= beta_final * (1 + 1e-12)) {
                    st = S_FINISH;
                } else {
                    beta *= factor;
                    if (beta < beta_final) beta = beta_final;
                    st = S_LEVEL;
                }
                break;
            case S_FINISH:
                // the last accepted iterate back to the caller's physical v
                // (left untouched when nothing was accepted; a coarse grid of
                // the continuation keeps it on the half spectrum)
                if (changed && v) STCHK(from_spec(ctx, ctx->vhat, v));
                ctx->beta = P.beta;
                rep->final_beta = beta;
                rep->final_gref = g0;
                rep->status = status;
                rep->n_iter = it;
                rep->final_J = J;
                rep->final_mismatch = mis;
                rep->final_grel = g0 > 0 ? gnorm / g0 : 0;
                rep->interps = ctx->interps - interps0;
                rep->alg_bytes = ctx->alg_bytes - alg0;
                rep->seconds_total = secs(t0);
                st = S_DONE;
                return REG_OK;
            case S_DONE:
                return REG_OK;
            }
        }
    }
};

// Runs the solvers to completion in rounds (one stream synchronisation per
// round). Returns the first HIP-level failure; per-problem outcomes are in
// each solver's status.
template <typename T>
reg_status run_solvers(Exec<T> &ex, std::vector<Solver> &S) {
    for (auto &s : S) {
        reg_status st = s.advance<T>();
        if (st != REG_OK) return st;
    }
    for (;;) {
        std::vector<Item> items;
        bool active = false;
        for (auto &s : S) {
            if (s.done()) continue;
            active = true;
            if (s.req.op != Op::NONE) items.push_back({s.ctx, s.req});
        }
        if (!active) break;
        auto t = clk::now();
        reg_status st = ex.round(items);
        if (st != REG_OK) return st;
        HIPCHK(S[0].ctx, hipStreamSynchronize(ex.stream));
        const double dt = secs(t);
        for (auto &s : S) {
            if (s.done()) continue;
            if (!s.ctx->prof.pending.empty()) s.ctx->prof.resolve();
            switch (s.req.op) {
            case Op::GRADIENT: s.rep->seconds_gradient += dt; break;
            case Op::MATVEC: s.rep->seconds_matvec += dt; break;
            case Op::OBJECTIVE: s.rep->seconds_objective += dt; break;
            default: s.rep->seconds_precond += dt; break;
            }
            st = s.advance<T>();
            if (st != REG_OK) return st;
        }
        if (ex.b && !ex.b->prof.pending.empty()) ex.b->prof.resolve();
    }
    // the last advance() of each problem queued its result transform
    HIPCHK(S[0].ctx, hipStreamSynchronize(ex.stream));
    return REG_OK;
}

// single heavy operation of one context (synchronises when it has scalars)
template <typename T>
reg_status single_op(reg_ctx *ctx, const Request &r) {
    Exec<T> ex(nullptr, ctx->stream);
    std::vector<Item> items{{ctx, r}};
    STCHK(ex.round(items));
    if (slots_of(r) > 0) {
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        if (!ctx->prof.pending.empty()) ctx->prof.resolve();
    }
    return REG_OK;
}

// The solve of one context over `levels` grids of its chain (grid
// continuation; levels = 1: this grid only). With start_hat the first iterate
// is already in ctx->vhat and v may be null (a coarse grid of the chain).
template <typename T>
reg_status solve_chain(reg_ctx *ctx, void *v, reg_report *rep, int levels, bool start_hat) {
    const auto t0 = clk::now();
    const int64_t fft3d0 = ctx->fft3d, lines0 = ctx->fft_lines;
    const double alg_start = ctx->alg_bytes;
    double alg_coarse = 0;  // the coarser grids' solves
    double beta_start = 0, gref_start = 0;
    if (levels > 1) {
        reg_ctx *c = ctx->coarse;
        if (!ctx->coarse_images) {
            // images restricted by spectral truncation
            STCHK(resample_fields<T>(ctx, c, 1, ctx->rhoT, c->rhoT));
            STCHK(resample_fields<T>(ctx, c, 1, ctx->rhoR, c->rhoR));
            STCHK(reduce<T>(c, c->rhoT, c->rhoR, c->N, 1, h3(c), 0));
            STCHK(fetch(c, 1));
            c->normTR2 = c->hres[0];
            c->have_images = true;
            c->coarse_images = false;
            ctx->coarse_images = true;
        }
        c->have_state = false;
        if (!start_hat) STCHK(to_spec(ctx, v, ctx->vhat));
        STCHK(resample_vec_hat(ctx, ctx->vhat, c, c->vhat));
        std::unique_ptr<reg_report> rc(new (std::nothrow) reg_report());
        if (!rc) return fail(ctx, REG_ENOMEM, "host allocation of a coarse-grid report");
        std::memset(rc.get(), 0, sizeof(reg_report));
        const reg_status sc = solve_chain<T>(c, nullptr, rc.get(), levels - 1, true);
        // a coarse grid whose line search stalled still hands on its last
        // accepted iterate; any other failure ends the solve
        if (sc != REG_OK && sc != REG_ELINESEARCH) return fail(ctx, sc, "coarse grid: " + c->err);
        rep->grid_levels = rc->grid_levels;
        for (int l = 0; l < rc->grid_levels; l++) {
            for (int j = 0; j < 3; j++) rep->level_n[l][j] = rc->level_n[l][j];
            rep->level_iters[l] = rc->level_iters[l];
            rep->level_matvecs[l] = rc->level_matvecs[l];
            rep->level_seconds[l] = rc->level_seconds[l];
            rep->level_mismatch[l] = rc->level_mismatch[l];
            rep->level_beta[l] = rc->level_beta[l];
        }
        // prolongation by spectral zero-padding
        STCHK(resample_vec_hat(c, c->vhat, ctx, ctx->vhat));
        beta_start = rc->final_beta;
        gref_start = rc->final_gref;
        alg_coarse = rc->alg_bytes;
        start_hat = true;
    }
    Exec<T> ex(nullptr, ctx->stream);
    std::vector<Solver> S(1);
    S[0].ctx = ctx;
    S[0].v = v;
    S[0].rep = rep;
    S[0].start_hat = start_hat;
    S[0].beta_start = beta_start;
    S[0].gref_start = gref_start;
    const reg_status st = run_solvers<T>(ex, S);
    ctx->beta = ctx->P.beta;
    const int l = rep->grid_levels < REG_MAXLEVELS ? rep->grid_levels : REG_MAXLEVELS - 1;
    for (int j = 0; j < 3; j++) rep->level_n[l][j] = ctx->P.n[j];
    rep->level_iters[l] = rep->n_iter;
    rep->level_matvecs[l] = rep->matvecs;
    rep->level_seconds[l] = rep->seconds_total;
    rep->level_mismatch[l] = rep->final_mismatch;
    rep->level_beta[l] = rep->final_beta;
    rep->grid_levels = l + 1;
    rep->fft3d = ctx->fft3d - fft3d0;
    rep->fft_lines = ctx->fft_lines - lines0;
    // wall clock and algorithmic bytes of everything above, every grid
    auto finish = [&]() {
        rep->seconds_total = secs(t0);
        rep->alg_bytes = ctx->alg_bytes - alg_start + alg_coarse;
    };
    if (st != REG_OK) {
        finish();
        return st;
    }
    // the map of the result and det grad y1 (on the caller's grid only)
    if (ctx->P.det_check && v && (S[0].status == REG_OK || S[0].status == REG_ELINESEARCH)) {
        STCHK(deformation_impl<T>(ctx, v, nullptr, &rep->det_min, &rep->det_max));
        if (S[0].status == REG_OK && !(rep->det_min > 0)) {
            finish();
            return fail(ctx, REG_ENONDIFFEO, "det grad y1 <= 0 at the result: the map is not a diffeomorphism");
        }
    }
    finish();
    return S[0].status;
}

template <typename T>
reg_status solve_one(reg_ctx *ctx, void *v, reg_report *rep) {
    return solve_chain<T>(ctx, v, rep, grid_count(&ctx->P), false);
}

template <typename T>
reg_status batch_solve(reg_batch *b, void *const *v, reg_report *reps) {
    Exec<T> ex(b, b->stream);
    std::vector<Solver> S(b->npairs);
    for (int i = 0; i < b->npairs; i++) {
        S[i].ctx = b->ctx[i];
        S[i].v = v[i];
        S[i].rep = &reps[i];
    }
    reg_status st = run_solvers<T>(ex, S);
    for (auto *c : b->ctx) c->beta = c->P.beta;
    for (int i = 0; i < b->npairs; i++) {
        reg_report *r = &reps[i];
        for (int j = 0; j < 3; j++) r->level_n[0][j] = b->ctx[i]->P.n[j];
        r->level_iters[0] = r->n_iter;
        r->level_matvecs[0] = r->matvecs;
        r->level_seconds[0] = r->seconds_total;
        r->level_mismatch[0] = r->final_mismatch;
        r->level_beta[0] = r->final_beta;
        r->grid_levels = 1;
    }
    if (st != REG_OK) return st;
    for (auto &s : S)
        if (s.status != REG_OK) return bfail(b, s.status, "pair " + std::to_string(&s - S.data()) + ": " + s.ctx->err);
    return REG_OK;
}

template <typename T>
reg_status batch_round(reg_batch *b, std::vector<Item> &items) {
    Exec<T> ex(b, b->stream);
    STCHK(ex.round(items));
    HIPCHK(items[0].ctx, hipStreamSynchronize(b->stream));
    for (auto &it : items)
        if (!it.ctx->prof.pending.empty()) it.ctx->prof.resolve();
    if (!b->prof.pending.empty()) b->prof.resolve();
    return REG_OK;
}

size_t batch_tables(const reg_params *pp, int32_t n, size_t *entries) {
    int ntmax = 0;
    for (int i = 0; i < n; i++) ntmax = std::max(ntmax, pp[i].nt);
    // per region: the steps of one round (state, incremental state, div v
    // interpolation and backward sweeps), one entry per problem each
    *entries = (size_t)n * (3 * (size_t)ntmax + 2);
    return align_up(sizeof(regk::PairStep) * *entries * (2 + reg_batch::kGraphs));
}

reg_status check_batch(const reg_params *pp, int32_t n, std::string *why) {
    if (!pp || n < 1 || n > 4096) {
        *why = "need 1 <= npairs <= 4096 parameter sets";
        return REG_EINVAL;
    }
    for (int i = 0; i < n; i++) {
        if (check_params(&pp[i], why) != REG_OK) {
            *why = "pair " + std::to_string(i) + ": " + *why;
            return REG_EINVAL;
        }
        if (pp[i].prec != pp[0].prec) {
            *why = "every pair of a batch needs the same prec";
            return REG_EINVAL;
        }
        if (grid_count(&pp[i]) > 1) {
            *why = "pair " + std::to_string(i) + ": grid continuation (grid_levels > 1) is a single-context solve";
            return REG_EINVAL;
        }
        if (pp[i].hessian) {
            *why = "pair " + std::to_string(i) + ": the full Newton Hessian (hessian = 1) is a single-context option";
            return REG_EINVAL;
        }
    }
    return REG_OK;
}

#define BATCH_OK(b)                                   \
    do {                                              \
        if (!(b)) return REG_EINVAL;                  \
        (b)->err.clear();                             \
    } while (0)

}  // namespace

// ====================================================================== ABI

extern "C" {

reg_status reg_gradient(reg_ctx *ctx, const void *v, void *g, double *J, double *mismatch, double *gnorm) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    NEED_DEV(ctx, g);
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    ctx->have_state = false;
    STCHK(to_spec(ctx, v, ctx->vhat));
    Request r{Op::GRADIENT, ctx->vhat, ctx->ghat, nullptr, false, false};
    STCHK(DISPATCH(ctx, single_op, ctx, r));
    STCHK(from_spec(ctx, ctx->ghat, g));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    scalars_to_J(ctx, J, mismatch);
    if (gnorm) *gnorm = std::sqrt(ctx->hres[3]);
    if (!std::isfinite(ctx->hres[1]) || !std::isfinite(ctx->hres[2]) || !std::isfinite(ctx->hres[3]))
        return fail(ctx, REG_ENONFINITE, "non-finite objective or gradient");
    ctx->have_state = true;
    return REG_OK;
}

reg_status reg_objective(reg_ctx *ctx, const void *v, double *J, double *mismatch) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v);
    if (!J || !mismatch) return fail(ctx, REG_EINVAL, "J and mismatch are required");
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    STCHK(to_spec(ctx, v, ctx->vthat));
    Request r{Op::OBJECTIVE, ctx->vthat, nullptr, nullptr, false, false};
    STCHK(DISPATCH(ctx, single_op, ctx, r));
    scalars_to_J(ctx, J, mismatch);
    if (!std::isfinite(*J)) return fail(ctx, REG_ENONFINITE, "non-finite objective");
    return REG_OK;
}

reg_status reg_hessian_matvec(reg_ctx *ctx, const void *vt, void *Hvt) {
    CTX_OK(ctx);
    NEED_DEV(ctx, vt);
    NEED_DEV(ctx, Hvt);
    if (!ctx->have_state) return fail(ctx, REG_EINVAL, "reg_gradient must be called first");
    STCHK(to_spec(ctx, vt, ctx->rhat));
    Request r{Op::MATVEC, ctx->rhat, ctx->qhat, nullptr, false, false};
    STCHK(DISPATCH(ctx, single_op, ctx, r));
    return from_spec(ctx, ctx->qhat, Hvt);
}

reg_status reg_solve(reg_ctx *ctx, void *v_inout, reg_report *rep) {
    CTX_OK(ctx);
    NEED_DEV(ctx, v_inout);
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    reg_report local;
    reg_report *r = rep ? rep : &local;
    std::memset(r, 0, sizeof(*r));
    ctx->have_state = false;
    reg_status st = DISPATCH(ctx, solve_one, ctx, v_inout, r);
    r->status = st;
    return st;
}

// ------------------------------------------------------------------ batch

reg_status reg_batch_workspace_size(const reg_params *per_pair, int32_t npairs, size_t *bytes) {
    std::string why;
    if (check_batch(per_pair, npairs, &why) != REG_OK || !bytes) return REG_EINVAL;
    size_t total = 0, entries = 0;
    for (int i = 0; i < npairs; i++) total += align_up(layout(&per_pair[i], nullptr, nullptr));
    total += batch_tables(per_pair, npairs, &entries);
    *bytes = total;
    return REG_OK;
}

reg_status reg_batch_create(const reg_params *per_pair, int32_t npairs, void *workspace, size_t bytes,
                            void *hip_stream, reg_batch **out) {
    if (!out) return REG_EINVAL;
    *out = nullptr;
    std::string why;
    if (check_batch(per_pair, npairs, &why) != REG_OK) {
        std::fprintf(stderr, "reg_batch_create: %s\n", why.c_str());
        return REG_EINVAL;
    }
    size_t need = 0;
    if (reg_batch_workspace_size(per_pair, npairs, &need) != REG_OK) return REG_EINVAL;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || !is_device_ptr(workspace)) return REG_EINVAL;
    if (bytes < need) return REG_ENOMEM;
    reg_batch *b = new (std::nothrow) reg_batch();
    if (!b) return REG_ENOMEM;
    b->npairs = npairs;
    b->prec = per_pair[0].prec;
    if (hip_stream) {
        b->stream = (hipStream_t)hip_stream;
    } else {
        // graphs cannot be captured on the null stream: use a stream of our
        // own (blocking, so it stays ordered with the null stream)
        if (hipStreamCreate(&b->stream) != hipSuccess) {
            (void)hipGetLastError();
            delete b;
            return REG_EHIP;
        }
        b->own_stream = true;
    }
    b->prof.stream = b->stream;
    char *base = (char *)workspace;
    size_t off = 0;
    reg_status st = REG_OK;
    for (int i = 0; i < npairs && st == REG_OK; i++) {
        const size_t sz = align_up(layout(&per_pair[i], nullptr, nullptr));
        reg_ctx *c = nullptr;
        st = reg_create(&per_pair[i], base + off, sz, b->stream, &c);
        if (st == REG_OK) b->ctx.push_back(c);
        off += sz;
        b->nt_max = std::max(b->nt_max, per_pair[i].nt);
    }
    size_t entries = 0;
    const size_t tab_bytes = batch_tables(per_pair, npairs, &entries);
    b->region = entries;
    b->dev_tab = (regk::PairStep *)(base + off);
    if (st == REG_OK && hipHostMalloc((void **)&b->host_tab, tab_bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        st = REG_EHIP;
    }
    if (st != REG_OK) {
        for (auto *c : b->ctx) reg_destroy(c);
        if (b->host_tab) (void)hipHostFree(b->host_tab);
        if (b->own_stream) (void)hipStreamDestroy(b->stream);
        delete b;
        return st;
    }
    *out = b;
    return REG_OK;
}

reg_status reg_batch_destroy(reg_batch *b) {
    if (!b) return REG_EINVAL;
    (void)hipStreamSynchronize(b->stream);
    for (auto &g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    for (auto *c : b->ctx) reg_destroy(c);
    b->prof.release();
    if (b->host_tab) (void)hipHostFree(b->host_tab);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
    return REG_OK;
}

const char *reg_batch_last_error(const reg_batch *b) { return b ? b->err.c_str() : "null batch"; }

reg_status reg_batch_ctx(reg_batch *b, int32_t pair, reg_ctx **ctx) {
    BATCH_OK(b);
    if (!ctx || pair < 0 || pair >= b->npairs) return bfail(b, REG_EINVAL, "pair out of range");
    *ctx = b->ctx[pair];
    return REG_OK;
}

reg_status reg_batch_set_launch(reg_batch *b, int32_t blocks, int32_t chunked, int32_t use_graph) {
    BATCH_OK(b);
    if (blocks != 0 && blocks < 8) return bfail(b, REG_EINVAL, "blocks must be 0 (autotune) or >= 8");
    if (chunked != 0 && chunked != 1) return bfail(b, REG_EINVAL, "chunked must be 0 or 1");
    b->fixed_blocks = blocks;
    b->fixed_chunked = chunked;
    b->use_graph = use_graph != 0;
    return REG_OK;
}

reg_status reg_batch_set_tile(reg_batch *b, int32_t tile1, int32_t tile2) {
    BATCH_OK(b);
    bool known = tile1 == 0 && tile2 == 0;
    for (int i = 0; i < regk::kBatchTileCount; i++)
        known = known || (regk::kBatchTiles[i][0] == tile1 && regk::kBatchTiles[i][1] == tile2);
    if (!known) return bfail(b, REG_EINVAL, "tile must be 0 x 0 (autotune) or one of 4x8, 2x8, 8x8, 4x4, 8x4");
    b->fixed_t1 = tile1;
    b->fixed_t2 = tile2;
    return REG_OK;
}

reg_status reg_batch_launch_info(reg_batch *b, int32_t mode, int32_t *blocks, int32_t *chunked, int32_t *variant,
                                 int32_t *tile1, int32_t *tile2, double *ms) {
    BATCH_OK(b);
    if (mode < 0 || mode > 2 || !blocks || !chunked || !variant || !tile1 || !tile2 || !ms)
        return bfail(b, REG_EINVAL, "bad launch query");
    *blocks = b->last[mode].blocks;
    *chunked = b->last[mode].chunked;
    *variant = b->last_variant[mode];
    *tile1 = b->last[mode].t1;
    *tile2 = b->last[mode].t2;
    *ms = b->last[mode].ms;
    return REG_OK;
}

reg_status reg_batch_stats(reg_batch *b, int64_t *batched_launches, int64_t *graph_captures, int64_t *graph_replays) {
    BATCH_OK(b);
    if (!batched_launches || !graph_captures || !graph_replays) return bfail(b, REG_EINVAL, "bad stats query");
    *batched_launches = b->launches;
    *graph_captures = b->captures;
    *graph_replays = b->replays;
    return REG_OK;
}

reg_status reg_batch_profile(reg_batch *b, int enable) {
    BATCH_OK(b);
    if (enable < 0) return bfail(b, REG_EINVAL, "reg_batch_profile: enable must be >= 0");
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, REG_EHIP, "hipStreamSynchronize failed");
    b->prof.resolve();
    if (enable) {
        b->prof.reset();
        b->prof.every = enable;
    }
    b->prof.on = enable != 0;
    for (auto *c : b->ctx) STCHK(reg_profile(c, enable));
    return REG_OK;
}

reg_status reg_batch_profile_read(reg_batch *b, int kind, int64_t *launches, double *ms) {
    BATCH_OK(b);
    if (kind < 0 || kind >= REG_K_COUNT || !launches || !ms) return bfail(b, REG_EINVAL, "bad profile query");
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, REG_EHIP, "hipStreamSynchronize failed");
    b->prof.resolve();
    *launches = b->prof.n[kind];
    *ms = b->prof.ms[kind];
    for (auto *c : b->ctx) {
        int64_t n = 0;
        double t = 0;
        STCHK(reg_profile_read(c, kind, &n, &t));
        *launches += n;
        *ms += t;
    }
    return REG_OK;
}

#define BATCH_ARRAY(b, arr)                                                                  \
    do {                                                                                     \
        if (!(arr)) return bfail((b), REG_EINVAL, #arr " is NULL");                          \
        for (int i_ = 0; i_ < (b)->npairs; i_++)                                             \
            if (!is_device_ptr((arr)[i_]))                                                   \
                return bfail((b), REG_EINVAL, #arr "[" + std::to_string(i_) + "] is not a device pointer"); \
    } while (0)

reg_status reg_batch_transport_forward(reg_batch *b, const void *const *v, const void *const *rho0, void *const *rho1) {
    BATCH_OK(b);
    BATCH_ARRAY(b, v);
    BATCH_ARRAY(b, rho0);
    BATCH_ARRAY(b, rho1);
    std::vector<Item> items;
    for (int i = 0; i < b->npairs; i++) {
        if (rho0[i] == rho1[i]) return bfail(b, REG_EINVAL, "rho1 must not alias rho0");
        items.push_back({b->ctx[i], Request{Op::FORWARD, v[i], rho1[i], rho0[i], false, false}});
    }
    return b->prec ? batch_round<double>(b, items) : batch_round<float>(b, items);
}

reg_status reg_batch_gradient(reg_batch *b, const void *const *v, void *const *g, double *J, double *mismatch,
                              double *gnorm) {
    BATCH_OK(b);
    BATCH_ARRAY(b, v);
    BATCH_ARRAY(b, g);
    std::vector<Item> items;
    for (int i = 0; i < b->npairs; i++) {
        reg_ctx *c = b->ctx[i];
        if (!c->have_images) return bfail(b, REG_EINVAL, "pair " + std::to_string(i) + ": images not set");
        c->have_state = false;
        STCHK(to_spec(c, v[i], c->vhat));
        items.push_back({c, Request{Op::GRADIENT, c->vhat, c->ghat, nullptr, false, false}});
    }
    STCHK(b->prec ? batch_round<double>(b, items) : batch_round<float>(b, items));
    for (int i = 0; i < b->npairs; i++) STCHK(from_spec(b->ctx[i], b->ctx[i]->ghat, g[i]));
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, REG_EHIP, "hipStreamSynchronize failed");
    for (int i = 0; i < b->npairs; i++) {
        reg_ctx *c = b->ctx[i];
        scalars_to_J(c, J ? &J[i] : nullptr, mismatch ? &mismatch[i] : nullptr);
        if (gnorm) gnorm[i] = std::sqrt(c->hres[3]);
        if (!std::isfinite(c->hres[1]) || !std::isfinite(c->hres[2]) || !std::isfinite(c->hres[3]))
            return bfail(b, REG_ENONFINITE, "pair " + std::to_string(i) + ": non-finite objective or gradient");
        c->have_state = true;
    }
    return REG_OK;
}

reg_status reg_batch_hessian_matvec(reg_batch *b, const void *const *vt, void *const *Hvt) {
    BATCH_OK(b);
    BATCH_ARRAY(b, vt);
    BATCH_ARRAY(b, Hvt);
    std::vector<Item> items;
    for (int i = 0; i < b->npairs; i++) {
        reg_ctx *c = b->ctx[i];
        if (!c->have_state) return bfail(b, REG_EINVAL, "reg_batch_gradient must be called first");
        STCHK(to_spec(c, vt[i], c->rhat));
        items.push_back({c, Request{Op::MATVEC, c->rhat, c->qhat, nullptr, false, false}});
    }
    STCHK(b->prec ? batch_round<double>(b, items) : batch_round<float>(b, items));
    for (int i = 0; i < b->npairs; i++) STCHK(from_spec(b->ctx[i], b->ctx[i]->qhat, Hvt[i]));
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, REG_EHIP, "hipStreamSynchronize failed");
    return REG_OK;
}

reg_status reg_batch_solve(reg_batch *b, void *const *v_inout, reg_report *reports) {
    BATCH_OK(b);
    BATCH_ARRAY(b, v_inout);
    if (!reports) return bfail(b, REG_EINVAL, "reports is NULL");
    for (int i = 0; i < b->npairs; i++) {
        reg_ctx *c = b->ctx[i];
        if (!c->have_images) return bfail(b, REG_EINVAL, "pair " + std::to_string(i) + ": images not set");
        c->have_state = false;
        std::memset(&reports[i], 0, sizeof(reg_report));
    }
    reg_status st = b->prec ? batch_solve<double>(b, v_inout, reports) : batch_solve<float>(b, v_inout, reports);
    return st;
}

}  // extern "C"
