// Launchers of the warm-start network kernels (net.hip), used by the host
// side in netapi.hip. Activations are BF16 (stored as uint16_t bit
// patterns), channel-last [point][channel]; every grid is a cube n^3 with
// points in C order (x3 fastest).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace regn {

// Convolution index maps, tap t = 9 a + 3 b + c with offsets d = (a-1, b-1, c-1):
//  FWD1: y[p] += W[t] x[p + d]                          (stride 1)
//  FWD2: y[p] += W[t] x[2p + d]     on a grid twice as fine (stride 2)
//  BWD1: y[q] += W[t]^T x[q - d]                        (backward data of FWD1)
//  BWD2: y[q] += W[t]^T x[(q - d)/2] when q - d is even  (backward data of FWD2)
enum { CONV_FWD1 = 0, CONV_FWD2 = 1, CONV_BWD1 = 2, CONV_BWD2 = 3 };

struct ConvArgs {
    const uint16_t *in;
    int in_cs;  // channel stride of in (>= cin, multiple of 4)
    int cin;    // GEMM K channels, multiple of 16 (<= 64)
    int n_in, n_out;
    const uint16_t *w;  // BF16 [27][cout][cin]
    int cout;           // GEMM N channels: 16, 32 or 64
    const float *bias;  // [cout_real] or null
    int relu;
    const uint16_t *add;  // optional: added before the mask, [p][add_cs]
    int add_cs;
    const uint16_t *mask;  // optional: zero where mask[p][c] <= 0 (ReLU backward)
    int mask_cs;
    uint16_t *out;  // BF16 [p][out_cs] (unless out_f32)
    int out_cs;
    float *out_f32;  // FP32 channel-first [cout_real][P] (network head)
    int cout_real;   // channels with a bias (and written to out_f32)
};

struct WgradArgs {
    const uint16_t *dz;  // output-side gradient [p][dz_cs], cout channels
    int dz_cs, cout;
    const uint16_t *x;  // layer input [q][x_cs], cin channels
    int x_cs, cin;
    int n_in, n_out;
    float *partials;       // [chunks][27][cout][cin]
    float *bias_partials;  // [chunks][cout]
};

hipError_t launch_conv(int mode, const ConvArgs &a, hipStream_t s);
int wgrad_chunks(int n_out);
hipError_t launch_wgrad(int mode, const WgradArgs &a, hipStream_t s);
hipError_t launch_wgrad_reduce(const float *partials, const float *bias_partials, int chunks, int cout, int cin,
                               int cout_real, int cin_real, float scale, float *dW, float *db, hipStream_t s);
hipError_t launch_up2(const uint16_t *x, int n_coarse, int C, uint16_t *y, hipStream_t s);
hipError_t launch_up2_bwd(const uint16_t *dy, int n_coarse, int C, const uint16_t *mask, int mask_cs, uint16_t *dz,
                          hipStream_t s);
hipError_t launch_mask(const uint16_t *src, int src_cs, long P, int C, const uint16_t *mask, int mask_cs, uint16_t *dz,
                       hipStream_t s);
hipError_t launch_pack_input(const float *a, const float *b, long P, uint16_t *x, hipStream_t s);
int mse_blocks(long P);
hipError_t launch_pack_head_grad(const float *dv, long P, float scale, uint16_t *dz, hipStream_t s);
hipError_t launch_mse(const float *v, const float *tgt, long P, double *partials, double *loss_acc, double scale,
                      uint16_t *dz, hipStream_t s);
hipError_t launch_adam(long n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s);
hipError_t launch_pack_weights(const float *W, int cout, int cin, int cout_pad, int cin_pad, uint16_t *fwd,
                               uint16_t *bwd, hipStream_t s);
hipError_t launch_unpack(const uint16_t *x, int cs, int C, long P, float *out, hipStream_t s);
hipError_t launch_fill_f32(long n, float v, float *x, hipStream_t s);
hipError_t launch_scale_f32(long n, float sc, float *x, hipStream_t s);

}  // namespace regn
