// C ABI of libreg (declared in include/reg.h): context creation over a
// caller-owned workspace and the single operators (interpolation, backtrace,
// spectral operators, transport solves, deformation). The reduced gradient,
// the Gauss-Newton matvec, the objective and the Gauss-Newton-Krylov driver
// live in solver.hip, which shares their execution with batches of problems.
#include "ctx.hpp"

using namespace regc;

namespace {

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
    alg_fields(ctx, 5.0 * ctx->P.nt);
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
        alg_fields(ctx, 5 + 3);  // div v interpolated, Heun factor
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
    alg_fields(ctx, (src ? 6.0 : 5.0) * nt);
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
    *bytes = total_size(p);
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
    if (bytes < total_size(p)) return REG_ENOMEM;
    if (!is_device_ptr(workspace)) return REG_EINVAL;
    reg_ctx *ctx = new (std::nothrow) reg_ctx();
    if (!ctx) return REG_ENOMEM;
    ctx->P = *p;
    ctx->beta = p->beta;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->prof.stream = ctx->stream;
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
    if (grid_count(p) > 1) {
        // the coarse-grid chain of the grid continuation, in the workspace
        // after this context's views
        const reg_params q = coarse_params(p);
        const size_t own = align_up(layout(p, nullptr, nullptr));
        const reg_status st = reg_create(&q, (char *)workspace + own, bytes - own, hip_stream, &ctx->coarse);
        if (st != REG_OK) {
            (void)hipHostFree(ctx->hres);
            delete ctx;
            return st;
        }
    }
    *out = ctx;
    return REG_OK;
}

reg_status reg_destroy(reg_ctx *ctx) {
    if (!ctx) return REG_EINVAL;
    if (ctx->coarse) reg_destroy(ctx->coarse);
    (void)hipStreamSynchronize(ctx->stream);
    ctx->prof.release();
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

reg_status reg_set_log(reg_ctx *ctx, reg_log_fn fn, void *user) {
    CTX_OK(ctx);
    for (reg_ctx *c = ctx; c; c = c->coarse) {
        c->log_fn = fn;
        c->log_user = user;
    }
    return REG_OK;
}

reg_status reg_set_solver(reg_ctx *ctx, const reg_params *p) {
    CTX_OK(ctx);
    std::string why;
    if (check_params(p, &why) != REG_OK) return fail(ctx, REG_EINVAL, why);
    if (p->n[0] != ctx->P.n[0] || p->n[1] != ctx->P.n[1] || p->n[2] != ctx->P.n[2] || p->nt != ctx->P.nt ||
        p->prec != ctx->P.prec)
        return fail(ctx, REG_EINVAL, "n, nt and prec are fixed at reg_create");
    int chain = 1;
    for (reg_ctx *c = ctx->coarse; c; c = c->coarse) chain++;
    if (p->hessian && !ctx->lamg)
        return fail(ctx, REG_EINVAL, "full Newton (hessian = 1) needs a context created with hessian = 1");
    if (!p->recompute_grad_rho && ctx->grho_levels == 1)
        return fail(ctx, REG_EINVAL, "a context created with recompute_grad_rho = 1 has no room for grad rho of "
                                     "every level");
    if (grid_count(p) > chain)
        return fail(ctx, REG_EINVAL, "grid_levels = " + std::to_string(p->grid_levels) + " exceeds the " +
                                         std::to_string(chain) + " grid(s) the workspace was laid out for");
    ctx->P = *p;
    ctx->beta = p->beta;
    ctx->have_state = false;
    reg_params q = *p;
    for (reg_ctx *c = ctx->coarse; c; c = c->coarse) {
        // coarser grids keep their own size and chain length
        const int32_t n[3] = {c->P.n[0], c->P.n[1], c->P.n[2]};
        q.grid_levels = q.grid_levels > 1 ? q.grid_levels - 1 : 0;
        c->P = q;
        for (int j = 0; j < 3; j++) c->P.n[j] = n[j];
        c->beta = q.beta;
        c->have_state = false;
    }
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
    ctx->coarse_images = false;
    return REG_OK;
}

reg_status reg_interp(reg_ctx *ctx, const void *f, const void *D, void *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, f);
    NEED_DEV(ctx, D);
    NEED_DEV(ctx, out);
    if (f == out) return fail(ctx, REG_EINVAL, "out must not alias f");
    ctx->interps++;
    alg_fields(ctx, 5);
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

reg_status reg_resample(reg_ctx *src, reg_ctx *dst, int ncomp, const void *in, void *out) {
    CTX_OK(src);
    if (!dst) return fail(src, REG_EINVAL, "dst is NULL");
    NEED_DEV(src, in);
    NEED_DEV(src, out);
    if (src->P.prec != dst->P.prec) return fail(src, REG_EINVAL, "src and dst must have the same precision");
    if (ncomp != 1 && ncomp != 3) return fail(src, REG_EINVAL, "ncomp must be 1 or 3");
    if (src == dst) return fail(src, REG_EINVAL, "src and dst must be different contexts");
    return src->P.prec ? resample_fields<double>(src, dst, ncomp, in, out) : resample_fields<float>(src, dst, ncomp, in, out);
}

reg_status reg_pad(reg_ctx *ctx, const int32_t m[3], const void *img, void *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, img);
    NEED_DEV(ctx, out);
    if (!m || m[0] < 1 || m[1] < 1 || m[2] < 1 || m[0] > ctx->g.n1 || m[1] > ctx->g.n2 || m[2] > ctx->g.n3)
        return fail(ctx, REG_EINVAL, "each m[j] must be in [1, n[j]]");
    if (img == out) return fail(ctx, REG_EINVAL, "out must not alias img");
    const int mm[3] = {m[0], m[1], m[2]};
    if (ctx->P.prec)
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_pad<double>(ctx->g, mm, CV<double>(img), V<double>(out), ctx->stream)));
    else
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_pad<float>(ctx->g, mm, CV<float>(img), V<float>(out), ctx->stream)));
    return REG_OK;
}

reg_status reg_crop(reg_ctx *ctx, const int32_t m[3], const void *field, void *out) {
    CTX_OK(ctx);
    NEED_DEV(ctx, field);
    NEED_DEV(ctx, out);
    if (!m || m[0] < 1 || m[1] < 1 || m[2] < 1 || m[0] > ctx->g.n1 || m[1] > ctx->g.n2 || m[2] > ctx->g.n3)
        return fail(ctx, REG_EINVAL, "each m[j] must be in [1, n[j]]");
    if (field == out) return fail(ctx, REG_EINVAL, "out must not alias field");
    const int mm[3] = {m[0], m[1], m[2]};
    if (ctx->P.prec)
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_crop<double>(ctx->g, mm, CV<double>(field), V<double>(out), ctx->stream)));
    else
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_crop<float>(ctx->g, mm, CV<float>(field), V<float>(out), ctx->stream)));
    return REG_OK;
}

reg_status reg_precond(reg_ctx *ctx, const void *r, void *z) {
    CTX_OK(ctx);
    NEED_DEV(ctx, r);
    NEED_DEV(ctx, z);
    STCHK(to_spec(ctx, r, ctx->rhat));
    STCHK(precond_hat(ctx, ctx->rhat, ctx->zhat));
    return from_spec(ctx, ctx->zhat, z);
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
    if (enable < 0) return fail(ctx, REG_EINVAL, "reg_profile: enable must be >= 0");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    if (enable) {
        ctx->prof.reset();
        ctx->prof.every = enable;
    }
    ctx->prof.on = enable != 0;
    return REG_OK;
}

reg_status reg_profile_read(reg_ctx *ctx, int kind, int64_t *launches, double *ms) {
    CTX_OK(ctx);
    if (kind < 0 || kind >= REG_K_COUNT || !launches || !ms) return fail(ctx, REG_EINVAL, "bad profile query");
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->prof.resolve();
    *launches = ctx->prof.n[kind];
    *ms = ctx->prof.ms[kind];
    return REG_OK;
}

}  // extern "C"
