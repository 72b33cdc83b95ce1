/*
 * reg.h -- C ABI of the MI355X (gfx950) semi-Lagrangian Gauss-Newton-Krylov
 * diffeomorphic registration library (method of Mang, Gholami and Biros,
 * "Distributed-memory large deformation diffeomorphic 3D image
 * registration", SC16).
 *
 * Problem (section II-B, eq. (2)): given a template rho_T and a reference
 * rho_R on the periodic box [0, 2*pi)^3, find a stationary velocity v that
 * minimises J(v) = 1/2 ||rho(1) - rho_R||^2 + beta/2 ||lap v||^2 subject to
 * the transport equation d_t rho + v . grad rho = 0, rho(0) = rho_T, and
 * optionally div v = 0.
 *
 * Conventions shared by every entry point
 *  - Grid: n[0] x n[1] x n[2] points x_i = 2*pi*i/n (section III-B1); arrays
 *    are C-order [n0][n1][n2], x3 fastest. A vector field is three such
 *    arrays back to back ([3][n0][n1][n2]).
 *  - Element types. Image-space fields (images, rho, lam, f, D, u, the
 *    outputs of reg_interp/reg_deriv/reg_grad/reg_div/reg_spectral) are float
 *    when params.prec == 0 and double when prec == 1. Velocity-space vectors
 *    (every argument named v, vt, g, Hvt, r, z, v_inout, and reg_dot's
 *    operands) are double in both modes: the H2 regulariser multiplies the
 *    representation error of v by |k|^4, which single precision cannot
 *    absorb on fine grids, so v, the gradient, the Krylov vectors and the 3D
 *    spectral operators on them are kept in double while the transport runs
 *    in the field type. Every pointer is a DEVICE pointer on the device that
 *    was current at reg_create, contiguous and aligned to its element size.
 *  - Semi-Lagrangian points are stored as displacements in cell units,
 *    D = (X - x)/h per axis, in the same element type.
 *  - Ownership: the caller owns every buffer it passes, including the
 *    workspace handed to reg_create (sized by reg_workspace_size). The
 *    library allocates no device memory; it keeps views into the workspace
 *    and a small pinned host buffer for scalar read-back.
 *  - Streams: all work is enqueued on the stream given to reg_create, in
 *    call order. Calls that return host scalars (reg_gradient, reg_solve,
 *    reg_deformation, reg_objective, reg_dot) synchronise that stream.
 *  - Errors: every call returns a reg_status; no C++ exception crosses the
 *    ABI. Arguments are checked before any kernel is launched; on REG_EINVAL
 *    nothing was enqueued. reg_last_error gives a message for the most recent
 *    failing call on a context.
 *  - Threading: one context per stream; a context is not re-entrant.
 *  - Inner products are the grid L2 ones, <u,w> = h1 h2 h3 sum u*w, and all
 *    reductions accumulate in double precision whatever the field type.
 */
#ifndef REG_H
#define REG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct reg_ctx reg_ctx;

typedef enum {
    REG_OK = 0,
    REG_EINVAL = 1,       /* bad argument or shape; nothing was enqueued        */
    REG_ENOMEM = 2,       /* workspace smaller than reg_workspace_size          */
    REG_EHIP = 3,         /* a HIP runtime call failed                          */
    REG_ENONFINITE = 4,   /* NaN/Inf met in an objective, norm or PCG product   */
    /* 5 is not used: a solve that runs out of Newton steps returns REG_OK and
     * reports stop_reason 2 */
    REG_ELINESEARCH = 6,  /* Armijo search found no acceptable step              */
    REG_ENONDIFFEO = 7,   /* params.det_check: det grad y1 <= 0 somewhere at the result */
    REG_ENOTIMPL = 8
} reg_status;

/* Discretisation and solver settings. reg_default_params fills the values of
 * the paper's runs (section IV-A3): beta = 1e-2, nt = 4, gradient tolerance
 * 1e-2, quadratic forcing, no continuation, no incompressibility. */
typedef struct {
    int32_t n[3];          /* grid; each even, 2^a 3^b 5^c, 8 <= n <= 1024        */
    int32_t nt;            /* time steps, >= 1                                    */
    double beta;           /* regularisation weight (> 0); first continuation level */
    double beta_final;     /* last continuation level; <= 0 means no continuation */
    double beta_factor;    /* continuation factor in (0, 1); default 0.1           */
    int32_t isochoric;     /* 1: enforce div v = 0 (Leray projection)              */
    int32_t prec;          /* 0: float fields, 1: double fields                    */
    double gtol;           /* stop a level at ||g|| <= gtol ||g0||                 */
    double mismatch_tol;   /* > 0: stop the solve at ||rho1-rhoR||/||rhoT-rhoR|| <= tol */
    int32_t max_newton;    /* Newton steps per continuation level                  */
    int32_t max_pcg;       /* PCG iterations per Newton step                       */
    int32_t max_ls;        /* Armijo trials per Newton step                        */
    int32_t forcing;       /* 0: eta = min(.5, r); 1: eta = min(.5, sqrt r); r = ||g||/||g0|| */
    double armijo_c1;      /* sufficient-decrease constant                         */
    double gnorm_ref;      /* > 0: stop a level at ||g|| <= gtol * gnorm_ref instead of
                            * gtol ||g0||, and use ||g||/gnorm_ref in the forcing term (an
                            * absolute reference, e.g. ||g(v=0)||, so that warm and cold
                            * starts run by the same rules); 0: ||g0||                */
    double gtol_level;     /* > 0: continuation levels above beta_final stop at
                            * ||g|| <= gtol_level * ref (the last level uses gtol); 0: gtol */
    int32_t grid_levels;   /* grid continuation: reg_solve first solves on grids coarsened by
                            * 2^(L-1), ..., 2 per axis, then on n (L = grid_levels, at most
                            * REG_MAXLEVELS; 0 or 1: n only). Every coarse grid must itself be a
                            * valid n. Fixes the workspace size: reg_set_solver may lower it only. */
    int32_t hessian;       /* 0: Gauss-Newton (the paper's runs, section IV-A3); 1: full Newton
                            * (eqs. (5a)-(5e) with both lam terms). 1 needs a workspace laid
                            * out for it (an extra adjoint history): reg_set_solver cannot
                            * switch a Gauss-Newton context to it. Single contexts only. */
    int32_t det_check;     /* 1: reg_solve computes det grad y1 of the result (eq. (1)) into the
                            * report and returns REG_ENONDIFFEO if its minimum is <= 0 */
    int32_t recompute_grad_rho; /* 0: keep grad rho^n of every time level (3 (nt+1) fields of the
                            * workspace); 1: keep one level and recompute grad rho^n by line FFTs
                            * wherever it is needed (section III-C1): the workspace shrinks by
                            * 3 nt fields, each transport step costs one more gradient. Fixes the
                            * workspace: reg_set_solver cannot turn it off. Not with hessian = 1. */
} reg_params;

#define REG_MAXIT 512
#define REG_MAXLEVELS 4

/* What reg_solve did, per accepted Newton step and in total. */
typedef struct {
    int32_t status;        /* the reg_status the solve returned                    */
    int32_t n_iter;        /* accepted Newton steps (entries below)                */
    int32_t matvecs, gradients, objectives;
    int32_t stop_reason;   /* 0 gradient tolerance, 1 mismatch, 2 step limit       */
    double J[REG_MAXIT], mismatch[REG_MAXIT], grel[REG_MAXIT], alpha[REG_MAXIT], beta[REG_MAXIT];
    int32_t pcg_iters[REG_MAXIT], ls_trials[REG_MAXIT];
    double final_J, final_mismatch, final_grel;
    double seconds_total;  /* host wall clock of the solve                         */
    /* wall clock of the executor rounds in which this problem ran a matvec,
     * a gradient, an objective, or only PCG vector work and preconditioning */
    double seconds_matvec, seconds_gradient, seconds_objective, seconds_precond;
    int64_t interps;       /* scalar field interpolations of n0*n1*n2 points       */
    double final_beta;     /* beta of the last continuation level worked on        */
    double final_gref;     /* that level's gradient reference (its g0)             */
    /* Grid continuation (params.grid_levels): one entry per grid solved,
     * coarsest first; the finest is the context's own grid, which every other
     * field above describes. Without grid continuation one entry. */
    int32_t grid_levels;
    int32_t level_n[REG_MAXLEVELS][3];
    int32_t level_iters[REG_MAXLEVELS], level_matvecs[REG_MAXLEVELS];
    double level_seconds[REG_MAXLEVELS], level_mismatch[REG_MAXLEVELS], level_beta[REG_MAXLEVELS];
    int32_t negative_curvature;  /* PCG runs ended by <p, H p> <= 0 (the step is the iterate so
                                  * far, or -M g at the first iteration)                  */
    int32_t descent_fallbacks;   /* Newton steps whose PCG step was no descent direction,
                                  * replaced by -M g before the line search                 */
    int64_t fft3d;         /* 3D transforms, one component each (context's grid)       */
    int64_t fft_lines;     /* line-FFT derivative passes, one field each               */
    double det_min, det_max;  /* det grad y1 of the result (params.det_check), else 0   */
    /* Algorithmic HBM bytes of the kernels the solve launched, on every grid:
     * each kernel's operands read and written once (transport steps, plans,
     * derivatives, 3D transforms, velocity-space passes, reductions). A model
     * from operand sizes and launch counts, not a counter reading; divided by
     * seconds_total it is the solve's average algorithmic bandwidth.        */
    double alg_bytes;
} reg_report;

/* Fills *p with the paper's defaults for an n^3 grid (section IV-A3). */
reg_status reg_default_params(reg_params *p);

/* Bytes of device workspace a context with these parameters needs. */
reg_status reg_workspace_size(const reg_params *p, size_t *bytes);

/* Creates a context over a caller-owned device workspace of at least
 * reg_workspace_size bytes (256-byte aligned). hip_stream is a hipStream_t
 * (NULL = the null stream). Uploads twiddle tables on that stream. */
reg_status reg_create(const reg_params *p, void *workspace, size_t bytes, void *hip_stream, reg_ctx **out);

/* Frees the context (not the workspace). */
reg_status reg_destroy(reg_ctx *ctx);

/* Message of the last failing call on ctx ("" if none); valid until the next call. */
const char *reg_last_error(const reg_ctx *ctx);

/* Changes beta (> 0) used by reg_gradient, reg_hessian_matvec, reg_precond. */
reg_status reg_set_beta(reg_ctx *ctx, double beta);

/* Progress log of reg_solve (and of this context's problem in
 * reg_batch_solve): after every accepted Newton step fn(json, user) receives
 * one line of JSON, {"n": [n0, n1, n2], "step": k, "beta": .., "J": ..,
 * "mismatch": .., "grel": ||g||/ref, "alpha": .., "pcg": .., "ls": ..,
 * "matvecs": .., "seconds": ..}, the string valid during the call only. With
 * grid continuation the coarser grids log too ("n" tells them apart). fn
 * runs on the calling host thread between GPU work and must not call the
 * library with this context. fn = NULL turns the log off. */
typedef void (*reg_log_fn)(const char *json, void *user);
reg_status reg_set_log(reg_ctx *ctx, reg_log_fn fn, void *user);

/* Replaces the solver settings of the context (beta and its continuation,
 * isochoric, tolerances, iteration limits, forcing, Armijo constant,
 * gnorm_ref); n, nt and prec must equal those given to reg_create.
 * Invalidates the cached state. */
reg_status reg_set_solver(reg_ctx *ctx, const reg_params *p);

/* Copies rho_T and rho_R (device fields) into the context and records
 * ||rho_T - rho_R|| for the relative mismatch. Invalidates cached state. */
reg_status reg_set_images(reg_ctx *ctx, const void *rho_T, const void *rho_R);

/* ---------------------------------------------------------------- kernels */

/* out(x_i) = f(x_i + h D_i) by periodic tricubic Lagrange interpolation on the
 * 4x4x4 stencil m-1..m+2 per axis, m = i + floor(D), t = D - floor(D)
 * (sections III-B2, III-C2). f, out: fields; D: vector field (cell units).
 * out must not alias f. */
reg_status reg_interp(reg_ctx *ctx, const void *f, const void *D, void *out);

/* For callers that cannot allocate device memory (code under stream capture
 * set-up, tight serving loops, harnesses that forbid hipMalloc): the same
 * interpolation as reg_interp, with no context, workspace or allocation.
 * prec: 0 float, 1 double; n: the grid (the sizes reg_create accepts, so at
 * most 1024^3 points); f, out: fields and D: displacement field, device
 * pointers on the current device, as for reg_interp (out must not alias f).
 * Enqueued on hip_stream (a hipStream_t, NULL = null stream); synchronises
 * that stream once, to read the floor bounds of D that choose the LDS tile
 * geometry. Scratch: a fixed 8 KiB device array per GPU (partial and final
 * floor bounds), held until the process ends and shared by every call on
 * that GPU: calls that overlap on one GPU race. Bad arguments return
 * REG_EINVAL with the reason on stderr; nothing is enqueued then. */
reg_status reg_interp_noalloc(int32_t prec, const int32_t n[3], const void *f, const void *D, void *out,
                              void *hip_stream);

/* RK2 departure points of the velocity sign*v for one step dt = 1/nt
 * (eq. (6)): X* = x - dt u(x), X = x - dt/2 (u(x) + u(X*)), u = sign*v,
 * returned as D = (X - x)/h. sign must be +1 or -1. D must not alias v. */
reg_status reg_backtrace(reg_ctx *ctx, const void *v, double sign, void *D);

/* Spectral derivative along axis (0, 1, 2) by line FFTs with symbol i k~
 * (Nyquist dropped) (section III-B1 and the line-FFT remark of III-C1). */
reg_status reg_deriv(reg_ctx *ctx, int axis, const void *u, void *du);

/* g = grad u (field-type vector) and d = div w (w a field-type vector),
 * spectral as above. */
reg_status reg_grad(reg_ctx *ctx, const void *u, void *g);
reg_status reg_div(reg_ctx *ctx, const void *w, void *d);

/* Even and projection operators on field-type data x by 3D real FFTs in the
 * field type:
 *  op 0: out = scale * lap^2 x            (symbol scale*|k|^4)
 *  op 1: out = (scale * lap^2)^-1 x       (identity on the k = 0 mode)
 *  op 2: out = Gaussian filter of width scale (radians), exp(-scale^2 |k|^2/2)
 *  op 3: out = P x, P = I - grad lap^-1 div (Leray; eq. (4))
 * ncomp is 1 or 3 (op 3 needs 3). out may alias x. */
reg_status reg_spectral(reg_ctx *ctx, int op, double scale, int ncomp, const void *x, void *out);

/* Spectral resampling of field-type data between the grids of two contexts
 * of the same precision (Fourier truncation from a finer grid or zero
 * padding to a coarser-to-finer one; the Nyquist planes of the smaller grid
 * are dropped; coefficients scaled by N_dst/N_src). Used for the multilevel
 * warm start. Work is enqueued on src's stream and uses both contexts'
 * spectral scratch. */
reg_status reg_resample(reg_ctx *src, reg_ctx *dst, int ncomp, const void *in, void *out);

/* Front end for images that are not periodic (section III-B1): zero padding.
 * img is an m[0] x m[1] x m[2] field-type array (C order, each m[j] <= n[j]);
 * out (the context's grid) receives it at offset (n[j] - m[j]) / 2 per axis
 * and zeros elsewhere. The paper then smooths the padded images with a
 * spectral Gaussian of one cell (reg_spectral, op 2, scale = the cell width) before the
 * registration. out must not alias img. */
reg_status reg_pad(reg_ctx *ctx, const int32_t m[3], const void *img, void *out);

/* The inverse of reg_pad: out (m[0] x m[1] x m[2]) = the centred block of the
 * field (the context's grid), e.g. to return rho(1) or a map component on the
 * image's own grid. out must not alias field. */
reg_status reg_crop(reg_ctx *ctx, const int32_t m[3], const void *field, void *out);

/* Spectral preconditioner of section III-A: z^ = r^/(beta |k|^4) for k != 0,
 * z^_0 = r^_0, followed by P when isochoric (double precision throughout).
 * z may alias r. */
reg_status reg_precond(reg_ctx *ctx, const void *r, void *z);

/* ------------------------------------------------------ transport solves */

/* State solve (eq. (2b)) with the RK2 semi-Lagrangian scheme (eqs. (6),(7)):
 * rho1 = rho(1) for rho(0) = rho0 under v. Does not disturb the state cached
 * by reg_gradient. */
reg_status reg_transport_forward(reg_ctx *ctx, const void *v, const void *rho0, void *rho1);

/* Adjoint solve (eq. (3)) backward from lam(1) = lam1 to lam0 = lam(0),
 * written in tau = 1 - t as transport by -v with source lam*div v (dropped
 * when isochoric). Does not disturb the cached state. */
reg_status reg_transport_adjoint(reg_ctx *ctx, const void *v, const void *lam1, void *lam0);

/* Reduced gradient g(v) = beta lap^2 v + P int_0^1 lam grad rho dt (eq. (4)),
 * plus J(v), the relative mismatch ||rho1 - rhoR|| / ||rhoT - rhoR|| and
 * ||g||. Needs reg_set_images. Caches the plans, the state history, grad rho
 * at every time level and div v for reg_hessian_matvec. Any of J, mismatch,
 * gnorm may be NULL. Synchronises. */
reg_status reg_gradient(reg_ctx *ctx, const void *v, void *g, double *J, double *mismatch, double *gnorm);

/* Objective and relative mismatch only (plan + state solve). Synchronises. */
reg_status reg_objective(reg_ctx *ctx, const void *v, double *J, double *mismatch);

/* Hessian matvec at the velocity of the last reg_gradient: Gauss-Newton
 * (eqs. (5a)-(5e) without the two adjoint terms, section II-B): incremental
 * state, incremental adjoint, H vt = beta lap^2 vt + P b~; with
 * params.hessian = 1 the full Newton matvec, whose incremental adjoint has
 * the source div(lam vt) and whose b~ adds int lam grad rho~ dt (lam: the
 * adjoint of that reg_gradient). */
reg_status reg_hessian_matvec(reg_ctx *ctx, const void *vt, void *Hvt);

/* Gauss-Newton-Krylov solve (section III-A): truncated PCG with the spectral
 * preconditioner and forcing eta, Armijo backtracking, beta continuation
 * from params.beta to params.beta_final. v_inout holds the initial velocity
 * (zero for a cold start) and receives the result; on REG_ELINESEARCH it
 * holds the last accepted iterate. rep may be NULL. Synchronises.
 *
 * With params.grid_levels = L > 1 the solve is continued over grids as well
 * as over beta (the paper's conclusion names slow convergence at small beta as
 * the open problem; a coarse grid makes each of its PCG iterations 8x
 * cheaper). The images and v_inout are restricted by spectral truncation to
 * the grid n/2^(L-1) (section III-B1); that grid is solved with the full
 * beta continuation and the same stopping rules; its velocity is prolonged by
 * spectral zero-padding to the next grid, whose solve resumes the
 * continuation at the beta level the coarser solve ended on, and keeps that
 * level's gradient reference g0 from the coarser grid (grid L2 norms
 * approximate the same continuous norm on every grid, so the grids together
 * stop where one grid would); and so on up to n. Every grid's work is
 * summarised in rep->level_*. */
reg_status reg_solve(reg_ctx *ctx, void *v_inout, reg_report *rep);

/* Deformation map of eq. (1) through u = y1 - x, transported like the state
 * (u^{n+1} = u^n(X) + h D), and min/max of det(I + grad u) over the grid.
 * u_or_null receives u (vector field) when not NULL. Synchronises. */
reg_status reg_deformation(reg_ctx *ctx, const void *v, void *u_or_null, double *detmin, double *detmax);

/* <a, b> of two velocity-space (double) vectors of ncomp components each
 * (h1 h2 h3 weights). */
reg_status reg_dot(reg_ctx *ctx, int ncomp, const void *a, const void *b, double *out);

/* ------------------------------------------------------------- batches */

/* A batch is a set of independent registration problems, each with its own
 * parameters and grid (mixed sizes allowed, one precision for all), solved
 * together on one stream. The work of all problems advances in rounds: every
 * semi-Lagrangian time step of all problems of a round goes out as one
 * persistent launch over a work list of (problem, tile) items -- every
 * problem whose departure box fits the 64 KB LDS tile (the rare others use
 * the single-problem direct gather in the same round) -- with the launch shape
 * (workgroup count, XCD dealing) chosen by an autotuner that times the
 * candidates on the first launch of each (step kind, box span, set of grid
 * sizes) and keeps the choice for the process. Hessian matvecs are replayed
 * from a captured HIP graph once the same problems repeat them with
 * unchanged plans. A problem's results are those of the single-problem entry
 * points on its own context (same kernels, same arguments). Problems are
 * independent (no communication); this is the data-parallel mode across
 * many image pairs. */
typedef struct reg_batch reg_batch;

/* Workspace bytes of a batch of npairs problems (per_pair[i] as for
 * reg_workspace_size; every prec equal). */
reg_status reg_batch_workspace_size(const reg_params *per_pair, int32_t npairs, size_t *bytes);

/* Creates the batch and one context per problem over a caller-owned device
 * workspace (256-byte aligned, reg_batch_workspace_size bytes). hip_stream
 * is the stream of all work; NULL makes the batch create a blocking stream
 * of its own (graphs cannot be captured on the null stream). Set each
 * problem's images through reg_batch_ctx + reg_set_images. */
reg_status reg_batch_create(const reg_params *per_pair, int32_t npairs, void *workspace, size_t bytes,
                            void *hip_stream, reg_batch **out);

/* Frees the batch and its contexts (not the workspace). */
reg_status reg_batch_destroy(reg_batch *b);

/* Message of the last failing batch call ("" if none). */
const char *reg_batch_last_error(const reg_batch *b);

/* The context of problem `pair` (owned by the batch; valid until
 * reg_batch_destroy). Every single-problem entry point works on it. */
reg_status reg_batch_ctx(reg_batch *b, int32_t pair, reg_ctx **ctx);

/* Launch configuration of the batched step kernel: blocks = 0 autotunes,
 * blocks >= 8 fixes the workgroup count; chunked = 1 deals the work list to
 * the 8 XCDs in contiguous chunks, 0 round-robin; use_graph = 0 runs every
 * matvec eagerly. Results do not depend on these settings. */
reg_status reg_batch_set_launch(reg_batch *b, int32_t blocks, int32_t chunked, int32_t use_graph);

/* Tile shape of the batched canonical launches: tile1 x tile2 x 64 output
 * points per workgroup of 64 tile2 threads, one of 4x8 (the default of the
 * single-problem kernels), 2x8, 8x8, 4x4, 8x4; 0 x 0 lets the launch tuner
 * pick it per launch (timing every shape whose box fits 64 KB and whose tiles
 * cover every problem's grid, with the workgroup counts). A fixed shape that
 * does not fit a launch falls back to the first that does. Results do not
 * depend on the shape. */
reg_status reg_batch_set_tile(reg_batch *b, int32_t tile1, int32_t tile2);

/* Workgroups, dealing, kernel variant, tile shape and tuned time (ms, 0 if
 * fixed) of the last batched launch of a step kind: mode 0
 * interpolation/state, 1 adjoint, 2 incremental state. A step takes one
 * batched launch per LDS box class of its problems: variant 1, 2, 4 for the
 * canonical box of that floor span, 0 for the generic box (4x8 tiles). */
reg_status reg_batch_launch_info(reg_batch *b, int32_t mode, int32_t *blocks, int32_t *chunked, int32_t *variant,
                                 int32_t *tile1, int32_t *tile2, double *ms);

/* Counters: batched step launches, graph captures, graph replays. */
reg_status reg_batch_stats(reg_batch *b, int64_t *batched_launches, int64_t *graph_captures, int64_t *graph_replays);

/* reg_profile / reg_profile_read over the batch: the batched launches and
 * graph replays plus every problem's own launches (enable as in
 * reg_profile). */
reg_status reg_batch_profile(reg_batch *b, int enable);
reg_status reg_batch_profile_read(reg_batch *b, int kind, int64_t *launches, double *ms);

/* Batched forms of reg_transport_forward, reg_gradient and
 * reg_hessian_matvec: array element i is problem i's argument (device
 * pointers; scalars in host arrays of npairs entries, which may be NULL for
 * J, mismatch, gnorm). Each synchronises the batch's stream. */
reg_status reg_batch_transport_forward(reg_batch *b, const void *const *v, const void *const *rho0, void *const *rho1);
reg_status reg_batch_gradient(reg_batch *b, const void *const *v, void *const *g, double *J, double *mismatch,
                              double *gnorm);
reg_status reg_batch_hessian_matvec(reg_batch *b, const void *const *vt, void *const *Hvt);

/* reg_solve for every problem of the batch (section III-A per problem):
 * v_inout[i] is problem i's initial velocity and result, reports[i] its
 * report (an array of npairs). Returns REG_OK when every problem returned
 * REG_OK, else the first failing problem's status (see reports[i].status;
 * the other problems still ran to completion). Synchronises. */
reg_status reg_batch_solve(reg_batch *b, void *const *v_inout, reg_report *reports);

/* ------------------------------------------------------ learned warm start */

/* A small network proposes the initial velocity of a solve (not part of the
 * paper, whose solver starts from v = 0 or the previous continuation level;
 * the solver decides whether to use it). It is a 3-level 3D convolutional
 * encoder-decoder on an n^3 grid (n = 64 in use): twelve 3x3x3 convolutions
 * with circular padding (channels 2->16->16, stride-2 16->32, 32->32,
 * stride-2 32->64, 64->64, 64->64, nearest upsampling, 64->32, concat with
 * the 32-channel encoder level -> 32, upsampling, 32->16, concat with the
 * 16-channel level -> 16, head 16->3), ReLU after every convolution but the
 * head. Input channels: (rho_T, rho_R) sampled on n^3; output: v [3][n^3].
 * The convolutions run on the matrix cores in BF16 with FP32 accumulation;
 * parameters are FP32 masters, in this order per layer: W[cout][cin][3][3][3]
 * (cross-correlation: y[o,p] = b[o] + sum W[o,c,a,b,d] x[c, s p + (a-1, b-1,
 * d-1)]) then b[cout]. Training minimises the mean squared error to target
 * velocities with Adam (beta1 0.9, beta2 0.999, eps 1e-8). */
typedef struct reg_net reg_net;

/* Number of FP32 parameters. */
reg_status reg_net_param_count(int64_t *count);

/* Device workspace of a network on an n^3 grid (n a multiple of 16, FFT
 * friendly, 16 <= n <= 256). It includes a single-precision context on n^3
 * used for spectral resampling in reg_warmstart. */
reg_status reg_net_workspace_size(int32_t n, size_t *bytes);

/* Creates the network over a caller-owned workspace (256-byte aligned);
 * parameters start at zero (set them with reg_net_set_params). */
reg_status reg_net_create(int32_t n, void *workspace, size_t bytes, void *hip_stream, reg_net **out);
reg_status reg_net_destroy(reg_net *net);
const char *reg_net_last_error(const reg_net *net);

/* Copies the parameters in from / out to a device array of
 * reg_net_param_count floats. Setting them resets the Adam moments. */
reg_status reg_net_set_params(reg_net *net, const float *params);
reg_status reg_net_get_params(reg_net *net, float *params);

/* v [3][n^3] (device, float) = network(rho_T, rho_R), images float n^3. */
reg_status reg_net_forward(reg_net *net, const float *rho_T, const float *rho_R, float *v);

/* After reg_net_forward: the output of convolution `layer` (0..11, after its
 * ReLU) as float [cout][m^3] on that layer's grid m (device). */
reg_status reg_net_activation(reg_net *net, int32_t layer, float *out);

/* Loss 1/(3 n^3) ||v - target||^2 of one sample and its gradient with
 * respect to every parameter (device float array, param_count entries).
 * Synchronises. */
reg_status reg_net_loss_grad(reg_net *net, const float *rho_T, const float *rho_R, const float *target, float *grad,
                             double *loss);

/* Backward pass of the last reg_net_forward for any loss L: dv = dL/dv
 * (device floats [3][n^3], the layout of reg_net_forward's v) in, grad =
 * dL/dparams (param_count device floats) out; the same kernels as
 * reg_net_loss_grad after its MSE head. REG_EINVAL without a preceding
 * reg_net_forward (set_params, loss_grad, train_step and warm starts reset
 * it). Synchronises. */
reg_status reg_net_backward(reg_net *net, const float *dv, float *grad);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) of the
 * parameters with the given gradient (param_count device floats, e.g. from
 * reg_net_backward), then the BF16 weight copies refreshed. Synchronises. */
reg_status reg_net_step(reg_net *net, const float *grad, double lr);

/* One Adam step on the mean loss over `batch` samples (host arrays of device
 * pointers to float n^3 images and [3][n^3] targets); returns the mean loss
 * before the step. Synchronises. */
reg_status reg_net_train_step(reg_net *net, int32_t batch, const float *const *rho_T, const float *const *rho_R,
                              const float *const *target, double lr, double *loss);

/* Warm start of a single-precision context with images set: its images are
 * resampled spectrally to the network grid, the network proposes v, v is
 * resampled to the context's grid (double, velocity space) and projected
 * when isochoric, and the proposal is kept only if min det(grad y1) > 0
 * (reg_deformation); otherwise v_out = 0 and *used_fallback = 1. detmin (may
 * be NULL) receives min det(grad y1) of the proposal. Synchronises. */
reg_status reg_warmstart(reg_ctx *ctx, reg_net *net, void *v_out, int32_t *used_fallback, double *detmin);

/* ------------------------------------------------------------- profiling */

/* Kernel families timed by the profiler. */
typedef enum {
    REG_K_INTERP = 0,     /* interpolation / state step: reads D (3 fields), gathers f, writes out  */
    REG_K_BACKTRACE = 1,  /* RK2 departure points                                                    */
    REG_K_ADJOINT = 2,    /* adjoint / incremental-adjoint step with the b accumulation              */
    REG_K_INCSTATE = 3,   /* fused incremental-state step                                            */
    REG_K_DEFORM = 4,     /* deformation-map step                                                    */
    REG_K_DERIV = 5,      /* line-FFT derivative passes                                              */
    REG_K_FFT3D = 6,      /* 3D real transform passes                                                */
    REG_K_SYMBOL = 7,     /* pointwise spectral symbols                                              */
    REG_K_REDUCE = 8,     /* double-precision reductions                                             */
    REG_K_VECTOR = 9,     /* vector updates and copies                                               */
    REG_K_GRAPH = 10,     /* replays of a batch's captured Hessian-matvec graph (whole graph)         */
    REG_K_COUNT = 11
} reg_kernel_kind;

/* enable = k >= 1 clears the counters and starts timing launches of the
 * context with a pair of HIP events on its stream: every launch for k = 1,
 * else the first of every k launches of each kernel family. 0 stops; a
 * negative value is REG_EINVAL. Each timed launch adds two event records,
 * which leave the GPU idle for a few microseconds, so long runs sample
 * (k = 16 adds well under 1% to a 256^3 solve). */
reg_status reg_profile(reg_ctx *ctx, int enable);

/* Number of timed launches and their summed GPU milliseconds for one
 * kernel family since profiling was enabled (synchronises the stream); the
 * average launch time is ms / launches. */
reg_status reg_profile_read(reg_ctx *ctx, int kind, int64_t *launches, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* REG_H */
