/* A registration driven from plain C through the library's ABI: device
 * memory from the HIP runtime, no Python or PyTorch. The 32^3 smooth case
 * (rho_T = (sin^2 x1 + sin^2 x2 + sin^2 x3) / 3, rho_R the same image shifted
 * by two cells along x1), FP64, nt = 4; prints the report's figures as one
 * line "status n_iter matvecs final_mismatch first_mismatch". */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "reg.h"

#define CHECK(call)                                                       \
    do {                                                                  \
        int st_ = (int)(call);                                            \
        if (st_ != 0) {                                                   \
            fprintf(stderr, "%s failed: %d\n", #call, st_);               \
            return 1;                                                     \
        }                                                                 \
    } while (0)

int main(void) {
    const int n = 32;
    const long N = (long)n * n * n;
    reg_params p;
    CHECK(reg_default_params(&p));
    p.n[0] = p.n[1] = p.n[2] = n;
    p.nt = 4;
    p.prec = 1;
    p.max_newton = 3;
    size_t bytes = 0;
    CHECK(reg_workspace_size(&p, &bytes));
    void *ws = NULL, *rhoT = NULL, *rhoR = NULL, *v = NULL;
    CHECK(hipMalloc(&ws, bytes));
    CHECK(hipMalloc(&rhoT, sizeof(double) * N));
    CHECK(hipMalloc(&rhoR, sizeof(double) * N));
    CHECK(hipMalloc(&v, sizeof(double) * 3 * N));
    double *hT = malloc(sizeof(double) * N), *hR = malloc(sizeof(double) * N);
    if (!hT || !hR) return 1;
    const double h = 8.0 * atan(1.0) / n;  /* 2 pi / n */
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++)
            for (int k = 0; k < n; k++) {
                const double s1 = sin(i * h), s2 = sin(j * h), s3 = sin(k * h);
                const double r1 = sin(((i + 2) % n) * h);
                hT[((long)i * n + j) * n + k] = (s1 * s1 + s2 * s2 + s3 * s3) / 3.0;
                hR[((long)i * n + j) * n + k] = (r1 * r1 + s2 * s2 + s3 * s3) / 3.0;
            }
    CHECK(hipMemcpy(rhoT, hT, sizeof(double) * N, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(rhoR, hR, sizeof(double) * N, hipMemcpyHostToDevice));
    CHECK(hipMemset(v, 0, sizeof(double) * 3 * N));
    reg_ctx *ctx = NULL;
    CHECK(reg_create(&p, ws, bytes, NULL, &ctx));
    CHECK(reg_set_images(ctx, rhoT, rhoR));
    reg_report rep;
    const reg_status st = reg_solve(ctx, v, &rep);
    printf("%d %d %d %.9f %.9f\n", (int)st, rep.n_iter, rep.matvecs, rep.final_mismatch, rep.mismatch[0]);
    CHECK(reg_destroy(ctx));
    CHECK(hipFree(ws));
    CHECK(hipFree(rhoT));
    CHECK(hipFree(rhoR));
    CHECK(hipFree(v));
    free(hT);
    free(hR);
    return st == REG_OK ? 0 : 2;
}
