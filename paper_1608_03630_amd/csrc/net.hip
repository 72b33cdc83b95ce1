// Kernels of the learned warm-start network: a 3-level 3D convolutional
// encoder-decoder (16/32/64 channels, 3x3x3 kernels, circular padding, skip
// concatenation) that maps the template and reference images on a 64^3 grid
// to an initial velocity. Not part of the paper's method: its Gauss-Newton
// solve starts from v = 0 (or the previous continuation level); this network
// only proposes the starting point; the solver decides whether to use it.
//
// Convolutions are implicit GEMMs on the matrix cores: for 16 output points
// (M) x 16 output channels (N), the K dimension runs over (tap, input
// channel) in chunks of 16 with v_mfma_f32_16x16x16_bf16 (BF16 operands,
// FP32 accumulation). Activations and activation gradients are BF16,
// channel-last ([point][channel], x3 fastest over points); weights are FP32
// masters with BF16 copies in the two layouts the forward and the
// backward-data GEMMs read. Lane layout of the MFMA (16x16x16, 64 lanes):
// lane l holds A[l%16][4(l/16)+i], B[4(l/16)+i][l%16] and
// D[4(l/16)+i][l%16], i = 0..3.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "net.hpp"

namespace regn {

namespace {

typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t f2bf(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

__device__ __forceinline__ int wrap(int x, int n) {
    x %= n;
    return x < 0 ? x + n : x;
}

// source point of output point (i, j, k) for tap offsets (d1, d2, d3); -1
// when the tap does not reach a source point (odd parity in CONV_BWD2)
template <int MODE>
__device__ __forceinline__ int source(int i, int j, int k, int d1, int d2, int d3, int n_out, int n_in) {
    if (MODE == CONV_FWD1) return (wrap(i + d1, n_in) * n_in + wrap(j + d2, n_in)) * n_in + wrap(k + d3, n_in);
    if (MODE == CONV_BWD1) return (wrap(i - d1, n_in) * n_in + wrap(j - d2, n_in)) * n_in + wrap(k - d3, n_in);
    if (MODE == CONV_FWD2)
        return (wrap(2 * i + d1, n_in) * n_in + wrap(2 * j + d2, n_in)) * n_in + wrap(2 * k + d3, n_in);
    // CONV_BWD2: fine output grid, coarse input grid
    const int y1 = wrap(i - d1, n_out), y2 = wrap(j - d2, n_out), y3 = wrap(k - d3, n_out);
    if ((y1 | y2 | y3) & 1) return -1;
    return ((y1 >> 1) * n_in + (y2 >> 1)) * n_in + (y3 >> 1);
}

// source coordinate along one axis of output coordinate i for the tap
// offset d, or -1 where the tap does not reach a source point (the axis
// form of source() above)
template <int MODE>
__device__ __forceinline__ int source_axis(int i, int d, int n_out, int n_in) {
    if (MODE == CONV_FWD1) return wrap(i + d, n_in);
    if (MODE == CONV_BWD1) return wrap(i - d, n_in);
    if (MODE == CONV_FWD2) return wrap(2 * i + d, n_in);
    const int y = wrap(i - d, n_out);  // CONV_BWD2: fine output grid, coarse input grid
    return (y & 1) ? -1 : (y >> 1);
}

// One wavefront: MB blocks of 16 consecutive output points x NB*16 output
// channels, starting at channel block blockIdx.y * NB (small grids split
// the channels over gridDim.y for more wavefronts). Each weight fragment
// feeds MB matrix products and each activation fragment NB, so a wavefront
// issues MB + NB fragment loads for MB * NB MFMAs per (tap, channel chunk).
template <int MODE, int NB, int MB>
__global__ __launch_bounds__(kThreads) void k_conv(ConvArgs a) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const long p0 = ((long)blockIdx.x * (kThreads / 64) + wave) * 16 * MB;
    const long P = (long)a.n_out * a.n_out * a.n_out;
    if (p0 >= P) return;  // whole wavefronts only (P is a multiple of 16 MB)
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n_out;
    // this lane's A-row point in each point block: its source coordinate per
    // axis for the offsets d = -1, 0, 1 (-1 where the tap does not reach a
    // source point), computed once instead of per tap
    int c1[MB][3], c2[MB][3], c3[MB][3];
#pragma unroll
    for (int m = 0; m < MB; m++) {
        const long pa = p0 + 16 * m + r;
        const int i = (int)(pa / ((long)n * n)), j = (int)((pa / n) % n), k = (int)(pa % n);
#pragma unroll
        for (int d = -1; d <= 1; d++) {
            c1[m][d + 1] = source_axis<MODE>(i, d, a.n_out, a.n_in);
            c2[m][d + 1] = source_axis<MODE>(j, d, a.n_out, a.n_in);
            c3[m][d + 1] = source_axis<MODE>(k, d, a.n_out, a.n_in);
        }
    }
    v4f acc[MB][NB];
#pragma unroll
    for (int m = 0; m < MB; m++)
#pragma unroll
        for (int b = 0; b < NB; b++) acc[m][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const uint16_t *__restrict__ in = a.in;
    const uint16_t *__restrict__ W = a.w;
    const int ccin = a.cin >> 4;
#pragma unroll
    for (int t = 0; t < 27; t++) {
        const int e1 = t / 9, e2 = (t / 3) % 3, e3 = t % 3;
        const uint16_t *src[MB];
        bool ok[MB];
#pragma unroll
        for (int m = 0; m < MB; m++) {
            const int x1 = c1[m][e1], x2 = c2[m][e2], x3 = c3[m][e3];
            ok[m] = (x1 | x2 | x3) >= 0;
            const int q = ok[m] ? (x1 * a.n_in + x2) * a.n_in + x3 : 0;
            src[m] = in + (long)q * a.in_cs + 4 * g;
        }
        const uint16_t *wt = W + ((long)t * a.cout + 16 * NB * blockIdx.y + r) * a.cin + 4 * g;
        int c = 0;
        if constexpr (MB == 1 && NB == 1) {
            // the small grids' form (one wavefront per SIMD, nothing else to
            // hide a fragment load behind): four channel chunks' loads in
            // flight before their matrix products, in the same order of
            // accumulation
            for (; c + 4 <= ccin; c += 4) {
                v4s av4[4], bv4[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    av4[q] = ok[0] ? *reinterpret_cast<const v4s *>(src[0] + 16 * (c + q)) : v4s{0, 0, 0, 0};
                    bv4[q] = *reinterpret_cast<const v4s *>(wt + 16 * (c + q));
                }
#pragma unroll
                for (int q = 0; q < 4; q++)
                    acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av4[q], bv4[q], acc[0][0], 0, 0, 0);
            }
        }
        for (; c < ccin; c++) {
            v4s av[MB], bv[NB];
#pragma unroll
            for (int m = 0; m < MB; m++)
                av[m] = ok[m] ? *reinterpret_cast<const v4s *>(src[m] + 16 * c) : v4s{0, 0, 0, 0};
#pragma unroll
            for (int b = 0; b < NB; b++) bv[b] = *reinterpret_cast<const v4s *>(wt + (long)b * 16 * a.cin + 16 * c);
#pragma unroll
            for (int m = 0; m < MB; m++)
#pragma unroll
                for (int b = 0; b < NB; b++)
                    acc[m][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[m], bv[b], acc[m][b], 0, 0, 0);
        }
    }
    // epilogue: lane holds D[4g+i][r] = (point p0+16m+4g+i, channel b*16+r)
#pragma unroll
    for (int m = 0; m < MB; m++)
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int co = (NB * blockIdx.y + b) * 16 + r;
            const float bias = (a.bias && co < a.cout_real) ? a.bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const long p = p0 + 16 * m + 4 * g + i;
                float v = acc[m][b][i] + bias;
                if (a.add) v += bf2f(a.add[p * a.add_cs + co]);
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.mask && !(bf2f(a.mask[p * a.mask_cs + co]) > 0.f)) v = 0.f;
                if (a.out_f32) {
                    if (co < a.cout_real) a.out_f32[(long)co * P + p] = v;
                } else {
                    a.out[p * a.out_cs + co] = f2bf(v);
                }
            }
        }
}

// The small-grid form with the taps split over the workgroup: its four
// wavefronts share one block of 16 output points and one 16-channel output
// block, each runs the taps t = w, w + 4, ... (7, 7, 7, 6 of them), and the
// four partial sums are added in a fixed order through LDS. On a 16^3 grid
// the general kernel leaves one wavefront per SIMD running 27 taps in a row,
// each waiting on its fragment loads; here there are four, with a quarter of
// the taps each.
template <int MODE>
__global__ __launch_bounds__(kThreads) void k_conv_ksplit(ConvArgs a) {
    __shared__ v4f red[kThreads / 64][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n_out;
    const long p0 = (long)blockIdx.x * 16;  // P is a multiple of 16: every block is whole
    const long pa = p0 + r;
    const int i = (int)(pa / ((long)n * n)), j = (int)((pa / n) % n), k = (int)(pa % n);
    int c1[3], c2[3], c3[3];
#pragma unroll
    for (int d = -1; d <= 1; d++) {
        c1[d + 1] = source_axis<MODE>(i, d, a.n_out, a.n_in);
        c2[d + 1] = source_axis<MODE>(j, d, a.n_out, a.n_in);
        c3[d + 1] = source_axis<MODE>(k, d, a.n_out, a.n_in);
    }
    v4f acc = v4f{0.f, 0.f, 0.f, 0.f};
    const int ccin = a.cin >> 4;
    for (int t = wave; t < 27; t += kThreads / 64) {
        const int x1 = c1[t / 9], x2 = c2[(t / 3) % 3], x3 = c3[t % 3];
        const bool ok = (x1 | x2 | x3) >= 0;
        const uint16_t *src = a.in + (long)(ok ? (x1 * a.n_in + x2) * a.n_in + x3 : 0) * a.in_cs + 4 * g;
        const uint16_t *wt = a.w + ((long)t * a.cout + 16 * (int)blockIdx.y + r) * a.cin + 4 * g;
        for (int c = 0; c < ccin; c++) {
            const v4s av = ok ? *reinterpret_cast<const v4s *>(src + 16 * c) : v4s{0, 0, 0, 0};
            const v4s bv = *reinterpret_cast<const v4s *>(wt + 16 * c);
            acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
        }
    }
    red[wave][lane] = acc;
    __syncthreads();
    if (wave != 0) return;
    v4f sum = red[0][lane];
#pragma unroll
    for (int w = 1; w < kThreads / 64; w++) sum += red[w][lane];
    // epilogue: lane holds D[4g+i][r] = (point p0+4g+i, channel blockIdx.y*16+r)
    const long P = (long)n * n * n;
    const int co = (int)blockIdx.y * 16 + r;
    const float bias = (a.bias && co < a.cout_real) ? a.bias[co] : 0.f;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const long p = p0 + 4 * g + q;
        float v = sum[q] + bias;
        if (a.add) v += bf2f(a.add[p * a.add_cs + co]);
        if (a.relu) v = fmaxf(v, 0.f);
        if (a.mask && !(bf2f(a.mask[p * a.mask_cs + co]) > 0.f)) v = 0.f;
        if (a.out_f32) {
            if (co < a.cout_real) a.out_f32[(long)co * P + p] = v;
        } else {
            a.out[p * a.out_cs + co] = f2bf(v);
        }
    }
}

// Backward data of a stride-2 convolution (CONV_BWD2) by output parity. An
// output point (2I + p1, 2J + p2, 2K + p3) of the fine grid receives only the
// taps whose offset has the parity of p along every axis (d = 0 for p = 0,
// d = +1 or -1 for p = 1: 1 to 8 of the 27 taps), whose sources are I (and
// I + 1 for d = -1). A wavefront takes 16 points of one parity class along
// x3 and all NB output channel blocks, and runs only those taps, in the
// order of the general kernel: the products it skips are those of zero
// activations, which add nothing to the general kernel's sums.
template <int NB>
__global__ __launch_bounds__(kThreads) void k_conv_bwd2(ConvArgs a) {
    const int lane = threadIdx.x & 63, g = lane >> 4, r = lane & 15;
    const int nc = a.n_in, nf = a.n_out, kb = nc / 16;
    long w = (long)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);  // wavefront index
    if (w >= 8L * nc * nc * kb) return;
    const int K0 = (int)(w % kb) * 16;
    w /= kb;
    const int J = (int)(w % nc);
    w /= nc;
    const int I = (int)(w % nc), cls = (int)(w / nc);
    const int p1 = cls >> 2, p2 = (cls >> 1) & 1, p3 = cls & 1;
    v4f acc[NB];
#pragma unroll
    for (int b = 0; b < NB; b++) acc[b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int ccin = a.cin >> 4;
    const int K = K0 + r;  // this lane's A-row point
    // taps per axis: d = 0 (source I) for even p, d = -1 (source I + 1) and
    // d = +1 (source I) for odd p, in ascending d
    for (int u1 = 0; u1 <= p1; u1++) {
        const int d1 = p1 ? 2 * u1 - 1 : 0, s1 = d1 < 0 ? (I + 1 == nc ? 0 : I + 1) : I;
        for (int u2 = 0; u2 <= p2; u2++) {
            const int d2 = p2 ? 2 * u2 - 1 : 0, s2 = d2 < 0 ? (J + 1 == nc ? 0 : J + 1) : J;
            for (int u3 = 0; u3 <= p3; u3++) {
                const int d3 = p3 ? 2 * u3 - 1 : 0, s3 = d3 < 0 ? (K + 1 == nc ? 0 : K + 1) : K;
                const int t = (d1 + 1) * 9 + (d2 + 1) * 3 + (d3 + 1);
                const uint16_t *src = a.in + ((long)(s1 * nc + s2) * nc + s3) * a.in_cs + 4 * g;
                const uint16_t *wt = a.w + ((long)t * a.cout + r) * a.cin + 4 * g;
                for (int c = 0; c < ccin; c++) {
                    const v4s av = *reinterpret_cast<const v4s *>(src + 16 * c);
#pragma unroll
                    for (int b = 0; b < NB; b++) {
                        const v4s bv = *reinterpret_cast<const v4s *>(wt + (long)b * 16 * a.cin + 16 * c);
                        acc[b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[b], 0, 0, 0);
                    }
                }
            }
        }
    }
    // epilogue: lane holds D[4g+i][r] = (point K0+4g+i of the class row, channel b*16+r)
    const long P = (long)nf * nf * nf;
    const long prow = ((long)(2 * I + p1) * nf + (2 * J + p2)) * nf + p3;
#pragma unroll
    for (int b = 0; b < NB; b++) {
        const int co = b * 16 + r;
        const float bias = (a.bias && co < a.cout_real) ? a.bias[co] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; i++) {
            const long p = prow + 2 * (K0 + 4 * g + i);
            float v = acc[b][i] + bias;
            if (a.add) v += bf2f(a.add[p * a.add_cs + co]);
            if (a.relu) v = fmaxf(v, 0.f);
            if (a.mask && !(bf2f(a.mask[p * a.mask_cs + co]) > 0.f)) v = 0.f;
            if (a.out_f32) {
                if (co < a.cout_real) a.out_f32[(long)co * P + p] = v;
            } else {
                a.out[p * a.out_cs + co] = f2bf(v);
            }
        }
    }
}

// Stride-1 convolutions (forward and backward data) as an LDS-tiled implicit
// GEMM. A workgroup owns a 4 x 4 x 16 tile of output points. For each chunk
// of 16 input channels it stages the tile's 6 x 6 x 18 halo in LDS
// ([halo point][16 channels], 20.7 KB) together with the chunk's weights of
// all 27 taps and its NB output channel blocks (13.8 KB per block), and runs
// all 27 taps from there: each of its
// four wavefronts takes four x3 rows of 16 points (one MFMA row block each)
// and NB output channel blocks starting at blockIdx.y * NB, reading per tap 4
// activation and NB weight fragments from LDS for 4 NB MFMAs.
constexpr int kCT1 = 4, kCT2 = 4, kCT3 = 16;                      // output tile
constexpr int kCH1 = kCT1 + 2, kCH2 = kCT2 + 2, kCH3 = kCT3 + 2;  // its halo
constexpr int kCHalo = kCH1 * kCH2 * kCH3;                        // 648 points

// Halo points are 32 bytes (16 channels), so the 16 points of one MFMA row
// block (consecutive h3) would put the same 8-byte channel group of points
// eight apart in the same LDS banks. The halo is staged by 16-byte direct
// loads, which move whole halves of a point, so the two halves trade places
// where bit 3 of h3 is set: points h3 and h3 + 8 then read different
// positions. The swizzle depends on h3 only, so reads of the same h3 in other
// (h1, h2) rows keep one base address.
__device__ __forceinline__ int halo_swap(int h3) { return (h3 >> 3) & 1; }
__device__ __forceinline__ int halo_group(int h3, int grp) { return grp ^ (halo_swap(h3) << 1); }
// The staged weights take 16-byte slots (the direct loads move whole pieces),
// so only the two halves of an output's 16 inputs can trade places: rows
// 8..15 store them swapped.
__device__ __forceinline__ int w_swap(int r) { return (r >> 3) & 1; }

template <int MODE, int NB>
__global__ __launch_bounds__(kThreads) void k_conv_tiled(ConvArgs a) {
    static_assert(MODE == CONV_FWD1 || MODE == CONV_BWD1, "stride-1 modes only");
    __shared__ __align__(16) uint16_t halo[kCHalo * 16];
    // weights of the chunk as [tap][block][output][16 inputs], padded to whole
    // rounds of 256 16-byte pieces
    constexpr int kWPieces = 27 * NB * 16 * 2, kWRounds = (kWPieces + kThreads - 1) / kThreads;
    __shared__ __align__(16) uint16_t wl[kWRounds * kThreads * 8];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n_out;  // == a.n_in
    const int nt3 = n / kCT3, nt2 = n / kCT2;
    const int t3 = (int)blockIdx.x % nt3, t2 = ((int)blockIdx.x / nt3) % nt2, t1 = (int)blockIdx.x / (nt3 * nt2);
    const int o1 = t1 * kCT1, o2 = t2 * kCT2, o3 = t3 * kCT3;
    const int cb0 = NB * (int)blockIdx.y;  // first output channel block
    const int sg = MODE == CONV_FWD1 ? 1 : -1;  // source = point + sg * d
    v4f acc[4][NB];
#pragma unroll
    for (int m = 0; m < 4; m++)
#pragma unroll
        for (int b = 0; b < NB; b++) acc[m][b] = v4f{0.f, 0.f, 0.f, 0.f};
    const int ccin = a.cin >> 4;
    for (int c = 0; c < ccin; c++) {
        // halo of channels [16c, 16c + 16): two 16-byte pieces per point
        constexpr int kPieces = (kCHalo * 2 + kThreads - 1) / kThreads;
        // weights: 16-byte piece e = ((t NB + b) 16 + r) 2 + sh holds eight
        // inputs of output channel (cb0 + b) 16 + r of tap t, loaded straight
        // into LDS (piece e at byte 16 e: a wavefront's 64 pieces land
        // contiguously from its wave-uniform base). Slot sh holds input half
        // sh ^ w_swap(r), which keeps the B fragments' 8-byte reads of rows r
        // and r + 8 in different banks.
#pragma unroll
        for (int u = 0; u < kWRounds; u++) {
            const int e = threadIdx.x + u * kThreads;
            if (e < kWPieces) {
                const int sh = e & 1, row = e >> 1;  // row = (t * NB + b) * 16 + r
                const int r16 = row & 15, tb = row >> 4, b = tb % NB, t = tb / NB;
                const uint16_t *src = a.w + ((long)t * a.cout + (cb0 + b) * 16 + r16) * a.cin + 16 * c +
                                      8 * (sh ^ w_swap(r16));
                uint16_t *dst = wl + 8 * (u * kThreads + 64 * wave);
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                                 (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
            }
        }
        // halo piece e (half sh of point hp = e / 2) goes straight into LDS at
        // byte 16 e, holding the point's channel half sh ^ halo_swap(h3)
#pragma unroll
        for (int u = 0; u < kPieces; u++) {
            const int e = threadIdx.x + u * kThreads;
            if (e < kCHalo * 2) {
                const int hp = e >> 1, sh = e & 1;
                const int h3 = hp % kCH3, h2 = (hp / kCH3) % kCH2, h1 = hp / (kCH3 * kCH2);
                const int x1 = wrap(o1 + h1 - 1, n), x2 = wrap(o2 + h2 - 1, n), x3 = wrap(o3 + h3 - 1, n);
                const long q = ((long)x1 * n + x2) * n + x3;
                const uint16_t *src = a.in + q * a.in_cs + 16 * c + 8 * (sh ^ halo_swap(h3));
                uint16_t *dst = halo + 8 * (u * kThreads + 64 * wave);
                __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void *)src,
                                                 (__attribute__((address_space(3))) void *)dst, 16, 0, 0);
            }
        }
        __builtin_amdgcn_s_waitcnt(0);  // the direct halo and weight loads have landed in LDS
        __syncthreads();
        // nine (d1, d2) rows of taps, the three d3 taps of a row unrolled
#pragma unroll 1
        for (int t12 = 0; t12 < 9; t12++)
#pragma unroll
        for (int e3 = 0; e3 < 3; e3++) {
            const int t = 3 * t12 + e3;
            const int d1 = t12 / 3 - 1, d2 = t12 % 3 - 1, d3 = e3 - 1;
            v4s bv[NB];
#pragma unroll
            for (int b = 0; b < NB; b++)
                bv[b] = *reinterpret_cast<const v4s *>(wl + ((t * NB + b) * 16 + r) * 16 + 4 * (g ^ (w_swap(r) << 1)));
#pragma unroll
            for (int m = 0; m < 4; m++) {
                const int pb = 4 * wave + m;  // x3 row (a1, a2) = (pb / 4, pb % 4)
                const int h1 = pb / kCT2 + 1 + sg * d1, h2 = pb % kCT2 + 1 + sg * d2, h3 = r + 1 + sg * d3;
                const v4s av =
                    *reinterpret_cast<const v4s *>(halo + ((h1 * kCH2 + h2) * kCH3 + h3) * 16 + 4 * halo_group(h3, g));
#pragma unroll
                for (int b = 0; b < NB; b++)
                    acc[m][b] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv[b], acc[m][b], 0, 0, 0);
            }
        }
        __syncthreads();  // the halo is restaged for the next chunk
    }
    // epilogue: lane holds D[4g+i][r] = (point 4g+i of row pb, channel (cb0+b)*16+r)
    const long P = (long)n * n * n;
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const int pb = 4 * wave + m;
        const long prow = ((long)(o1 + pb / kCT2) * n + o2 + pb % kCT2) * n + o3;
#pragma unroll
        for (int b = 0; b < NB; b++) {
            const int co = (cb0 + b) * 16 + r;
            const float bias = (a.bias && co < a.cout_real) ? a.bias[co] : 0.f;
#pragma unroll
            for (int i = 0; i < 4; i++) {
                const long p = prow + 4 * g + i;
                float v = acc[m][b][i] + bias;
                if (a.add) v += bf2f(a.add[p * a.add_cs + co]);
                if (a.relu) v = fmaxf(v, 0.f);
                if (a.mask && !(bf2f(a.mask[p * a.mask_cs + co]) > 0.f)) v = 0.f;
                if (a.out_f32) {
                    if (co < a.cout_real) a.out_f32[(long)co * P + p] = v;
                } else {
                    a.out[p * a.out_cs + co] = f2bf(v);
                }
            }
        }
    }
}

// Weight gradient partials: one workgroup per (chunk of wgrad_chunk(P) points, tap)
// forms sum_p dz[p][co] x[src(p, t)][ci] for every (co, ci) tile with
// v_mfma_f32_16x16x32_bf16 (K = points). Slices of kSlice points are staged
// transposed ([channel][point], row pitch kPitch) so that each lane's 8-point
// fragment is one 16-byte LDS read. The centre-tap workgroups also sum dz
// over their points (bias gradient).
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int kSlice = 64;
// points per weight-gradient workgroup: 2048 on 64^3 and finer grids, fewer
// on coarse ones so that they still spread over the GPU
__host__ __device__ inline int wgrad_chunk(long P) { return P >= 262144 ? 2048 : P >= 32768 ? 512 : 128; }
constexpr int kPitch = kSlice + 8;  // 144-byte rows: 16-byte aligned fragments

template <int MODE>
__global__ __launch_bounds__(kThreads) void k_wgrad(WgradArgs a) {
    __shared__ __align__(16) uint16_t sdz[64 * kPitch];
    __shared__ __align__(16) uint16_t sx[64 * kPitch];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int t = blockIdx.y;
    const int d1 = t / 9 - 1, d2 = (t / 3) % 3 - 1, d3 = t % 3 - 1;
    const int n = a.n_out;
    const long P = (long)n * n * n;
    const int cb = a.cout >> 4, ib = a.cin >> 4;
    const int tiles = cb * ib;  // <= 16: at most 4 per wavefront
    const int q4o = a.cout >> 2, q4i = a.cin >> 2;
    v4f acc[4];
#pragma unroll
    for (int u = 0; u < 4; u++) acc[u] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    const int chunk = wgrad_chunk(P);
    const long base = (long)blockIdx.x * chunk;
    for (int sl = 0; sl < chunk / kSlice; sl++) {
        const long s0 = base + (long)sl * kSlice;
        if (s0 >= P) break;
        for (int e = threadIdx.x; e < kSlice * q4o; e += kThreads) {
            const int pp = e / q4o, c = (e - pp * q4o) * 4;
            const v4s v = *reinterpret_cast<const v4s *>(a.dz + (s0 + pp) * a.dz_cs + c);
#pragma unroll
            for (int i = 0; i < 4; i++) sdz[(c + i) * kPitch + pp] = (uint16_t)v[i];
        }
        for (int e = threadIdx.x; e < kSlice * q4i; e += kThreads) {
            const int pp = e / q4i, c = (e - pp * q4i) * 4;
            const long p = s0 + pp;
            const int i1 = (int)(p / ((long)n * n)), i2 = (int)((p / n) % n), i3 = (int)(p % n);
            const int q = source<MODE>(i1, i2, i3, d1, d2, d3, a.n_out, a.n_in);
            const v4s v = *reinterpret_cast<const v4s *>(a.x + (long)q * a.x_cs + c);
#pragma unroll
            for (int i = 0; i < 4; i++) sx[(c + i) * kPitch + pp] = (uint16_t)v[i];
        }
        __syncthreads();
        if (t == 13 && threadIdx.x < a.cout)
            for (int pp = 0; pp < kSlice; pp++) bsum += bf2f(sdz[threadIdx.x * kPitch + pp]);
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int tile = wave + 4 * u;
            if (tile >= tiles) continue;
            const int co0 = (tile / ib) * 16, ci0 = (tile % ib) * 16;
#pragma unroll
            for (int kk = 0; kk < kSlice; kk += 32) {
                const v8s av = *reinterpret_cast<const v8s *>(sdz + (co0 + r) * kPitch + kk + 8 * g);
                const v8s bv = *reinterpret_cast<const v8s *>(sx + (ci0 + r) * kPitch + kk + 8 * g);
                acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av),
                                                                 __builtin_bit_cast(v8bf, bv), acc[u], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // partials[chunk][t][co][ci]
    float *out = a.partials + ((long)blockIdx.x * 27 + t) * a.cout * a.cin;
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const int tile = wave + 4 * u;
        if (tile >= tiles) continue;
        const int co0 = (tile / ib) * 16, ci0 = (tile % ib) * 16;
#pragma unroll
        for (int i = 0; i < 4; i++) out[(co0 + 4 * g + i) * a.cin + ci0 + r] = acc[u][i];
    }
    if (t == 13 && threadIdx.x < a.cout) a.bias_partials[(long)blockIdx.x * a.cout + threadIdx.x] = bsum;
}

// Weight gradients of stride-1 layers on 32^3 and finer grids, tiled like
// k_conv_tiled. A workgroup owns one block of 16 input channels
// (blockIdx.y), the nine taps of one x1 offset d1 = blockIdx.z - 1 and the
// wgrad_chunk(P) / 256 consecutive 4x4x16 tiles of its chunk. Per tile it
// stages the output-side gradient of all cout channels ([channel][point],
// the point order of the K dimension) and the four x1 planes of the layer
// input's 6x6x18 halo that its taps reach, for its 16 channels
// ([channel][h1][h2][h3]), once, then forms the products of its taps from
// LDS with v_mfma_f32_16x16x32_bf16 (K = the tile's 256 points, 32 at a
// time); each wavefront keeps the accumulators of its taps (9 d1 + wave +
// 4 u) across the chunk's tiles. Splitting the taps over three workgroups
// triples the workgroups of a launch (a 64^3 layer has only 128 chunks). A tap's x3 offset makes its 8-point input fragment start
// 0, 1 or 2 elements into an aligned 16-element window read as two 16-byte
// LDS loads; the odd case is cut out with funnel shifts. The partials and
// the bias partials have the layout of k_wgrad's.
constexpr int kWTile = kCT1 * kCT2 * kCT3;  // 256 points
constexpr int kWPitchZ = kWTile + 8;        // dz rows: 132 dwords, 4 mod 32 (conflict-free fragments)
constexpr int kWRowX = 24;                  // halo x3 rows: 18 used of 24 (the 16-element windows)
constexpr int kWPitchX = kCH1 * kCH2 * kWRowX + 8;  // per channel: 436 dwords, 4 mod 32

typedef int v4i __attribute__((ext_vector_type(4)));

template <int NCB>
__global__ __launch_bounds__(kThreads) void k_wgrad_tiled(WgradArgs a) {
    __shared__ __align__(16) uint16_t sdz[NCB * 16 * kWPitchZ];
    __shared__ __align__(16) uint16_t sx[16 * kWPitchX];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int g = lane >> 4, r = lane & 15;
    const int n = a.n_out;  // == a.n_in
    const long P = (long)n * n * n;
    const int nt3 = n / kCT3, nt2 = n / kCT2;
    const int tpc = wgrad_chunk(P) / kWTile;  // tiles per chunk
    const int cout = NCB * 16, ci0 = 16 * (int)blockIdx.y;
    const int z = (int)blockIdx.z;  // d1 + 1
    v4f acc[3][NCB];
#pragma unroll
    for (int u = 0; u < 3; u++)
#pragma unroll
        for (int b = 0; b < NCB; b++) acc[u][b] = v4f{0.f, 0.f, 0.f, 0.f};
    float bsum = 0.f;
    for (int ti = 0; ti < tpc; ti++) {
        const int tile = (int)blockIdx.x * tpc + ti;
        const int t3 = tile % nt3, t2 = (tile / nt3) % nt2, t1 = tile / (nt3 * nt2);
        const int o1 = t1 * kCT1, o2 = t2 * kCT2, o3 = t3 * kCT3;
        // output-side gradient: points pp, pp + 1 (pp = (4 a1 + a2) 16 + a3,
        // a3 even) of 4 channels a thread, transposed two points per 32-bit
        // LDS store
        // (the channel group is the slow index: a wavefront's stores then
        // fill consecutive dwords of one channel row)
        for (int e = threadIdx.x; e < kWTile / 2 * NCB * 4; e += kThreads) {
            const int pp = 2 * (e % (kWTile / 2)), c = (e / (kWTile / 2)) * 4;
            const int a1 = pp >> 6, a2 = (pp >> 4) & 3, a3 = pp & 15;
            const long p = ((long)(o1 + a1) * n + o2 + a2) * n + o3 + a3;
            const v4s v0 = *reinterpret_cast<const v4s *>(a.dz + p * a.dz_cs + c);
            const v4s v1 = *reinterpret_cast<const v4s *>(a.dz + (p + 1) * a.dz_cs + c);
#pragma unroll
            for (int i = 0; i < 4; i++)
                *reinterpret_cast<uint32_t *>(sdz + (c + i) * kWPitchZ + pp) =
                    (uint32_t)(uint16_t)v0[i] | ((uint32_t)(uint16_t)v1[i] << 16);
        }
        // halo planes h1 = z .. z + 3 of channels [ci0, ci0 + 16): points h3,
        // h3 + 1 (h3 even) of 8 channels a thread, two points per 32-bit store
        // (the channel half is the slow index, for the same reason)
        constexpr int kXPairs = kCT1 * kCH2 * (kCH3 / 2);
        for (int e = threadIdx.x; e < kXPairs * 2; e += kThreads) {
            const int hp2 = e % kXPairs, half = e / kXPairs;
            const int h3 = 2 * (hp2 % (kCH3 / 2)), h2 = (hp2 / (kCH3 / 2)) % kCH2, h1 = z + hp2 / ((kCH3 / 2) * kCH2);
            const int x1 = wrap(o1 + h1 - 1, n), x2 = wrap(o2 + h2 - 1, n);
            const int x3a = wrap(o3 + h3 - 1, n), x3b = wrap(o3 + h3, n);
            const long q = ((long)x1 * n + x2) * n;
            const v8s v0 = *reinterpret_cast<const v8s *>(a.x + (q + x3a) * a.x_cs + ci0 + 8 * half);
            const v8s v1 = *reinterpret_cast<const v8s *>(a.x + (q + x3b) * a.x_cs + ci0 + 8 * half);
            const int row = (h1 * kCH2 + h2) * kWRowX + h3;
#pragma unroll
            for (int i = 0; i < 8; i++)
                *reinterpret_cast<uint32_t *>(sx + (8 * half + i) * kWPitchX + row) =
                    (uint32_t)(uint16_t)v0[i] | ((uint32_t)(uint16_t)v1[i] << 16);
        }
        __syncthreads();
        if (blockIdx.y == 0 && z == 0 && threadIdx.x < cout) {
            const v8s *zr = reinterpret_cast<const v8s *>(sdz + threadIdx.x * kWPitchZ);
            for (int k = 0; k < kWTile / 8; k++) {
                const v8s z = zr[k];
#pragma unroll
                for (int i = 0; i < 8; i++) bsum += bf2f((uint16_t)z[i]);
            }
        }
        // K chunk m: x3 rows pb = 2m + (g >> 1) of the tile, points 8 (g & 1) .. + 7
#pragma unroll 1
        for (int m = 0; m < kWTile / 32; m++) {
            v8s av[NCB];
#pragma unroll
            for (int b = 0; b < NCB; b++)
                av[b] = *reinterpret_cast<const v8s *>(sdz + (16 * b + r) * kWPitchZ + 32 * m + 8 * g);
            const int pb = 2 * m + (g >> 1);
            const int a1 = pb >> 2, a2 = pb & 3;
#pragma unroll
            for (int u = 0; u < 3; u++) {
                const int tl = wave + 4 * u;  // tap within the d1 plane
                if (tl >= 9) continue;
                const int d1 = z - 1, d2 = tl / 3 - 1, sh = tl % 3;  // sh = 1 + d3
                const v4i *w = reinterpret_cast<const v4i *>(
                    sx + r * kWPitchX + ((a1 + 1 + d1) * kCH2 + a2 + 1 + d2) * kWRowX + 8 * (g & 1));
                const v4i w0 = w[0], w1 = w[1];
                v4i bx;
                if (sh == 0) {
                    bx = w0;
                } else if (sh == 2) {
                    bx = v4i{w0[1], w0[2], w0[3], w1[0]};
                } else {
                    bx = v4i{(int)__builtin_amdgcn_alignbit(w0[1], w0[0], 16),
                             (int)__builtin_amdgcn_alignbit(w0[2], w0[1], 16),
                             (int)__builtin_amdgcn_alignbit(w0[3], w0[2], 16),
                             (int)__builtin_amdgcn_alignbit(w1[0], w0[3], 16)};
                }
#pragma unroll
                for (int b = 0; b < NCB; b++)
                    acc[u][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, av[b]),
                                                                        __builtin_bit_cast(v8bf, bx), acc[u][b], 0, 0,
                                                                        0);
            }
        }
        __syncthreads();  // both buffers are restaged for the next tile
    }
    // partials[chunk][t][co][ci]: lane holds D[4 g + i][r] = (co 16 b + 4 g + i, ci ci0 + r)
#pragma unroll
    for (int u = 0; u < 3; u++) {
        const int tl = wave + 4 * u;
        if (tl >= 9) continue;
        const int t = 9 * z + tl;
        float *out = a.partials + ((long)blockIdx.x * 27 + t) * a.cout * a.cin;
#pragma unroll
        for (int b = 0; b < NCB; b++)
#pragma unroll
            for (int i = 0; i < 4; i++) out[(16 * b + 4 * g + i) * a.cin + ci0 + r] = acc[u][b][i];
    }
    if (blockIdx.y == 0 && z == 0 && threadIdx.x < cout)
        a.bias_partials[(long)blockIdx.x * a.cout + threadIdx.x] = bsum;
}

// dW[co][ci][t] += scale * sum over chunks and db[co] += scale * sum over
// chunks; real channels only. A workgroup sums 16 consecutive outputs
// (e = (t, co, ci), ci fastest, then the biases) over all chunks: thread
// (slice, j) adds chunks slice, slice + 16, ... of output j, and the 16
// slice sums are added in a fixed order, so the result is deterministic.
constexpr int kRedW = 16, kRedS = kThreads / kRedW;  // outputs x chunk slices per workgroup

__global__ __launch_bounds__(kThreads) void k_wgrad_reduce(const float *__restrict__ partials,
                                                           const float *__restrict__ bias_partials, int chunks,
                                                           int cout, int cin, int cout_real, int cin_real, float scale,
                                                           float *__restrict__ dW, float *__restrict__ db) {
    __shared__ float red[kRedS][kRedW + 1];
    const int j = threadIdx.x % kRedW, sl = threadIdx.x / kRedW;
    const int e = blockIdx.x * kRedW + j;
    const int nw = cout_real * cin_real * 27;
    float s = 0.f;
    if (e < nw) {
        const int ci = e % cin_real, co = (e / cin_real) % cout_real, t = e / (cin_real * cout_real);
        const long stride = 27L * cout * cin;
        const float *p = partials + ((long)t * cout + co) * cin + ci;
        for (int c = sl; c < chunks; c += kRedS) s += p[c * stride];
    } else if (e < nw + cout_real) {
        const int co = e - nw;
        for (int c = sl; c < chunks; c += kRedS) s += bias_partials[(long)c * cout + co];
    }
    red[sl][j] = s;
    __syncthreads();
    if (sl == 0 && e < nw + cout_real) {
        float tot = 0.f;
        for (int k = 0; k < kRedS; k++) tot += red[k][j];
        if (e < nw) {
            const int ci = e % cin_real, co = (e / cin_real) % cout_real, t = e / (cin_real * cout_real);
            dW[((long)co * cin_real + ci) * 27 + t] += scale * tot;
        } else {
            db[e - nw] += scale * tot;
        }
    }
}

// fine[q][c] = coarse[q/2][c] (nearest upsampling by 2 per axis)
__global__ __launch_bounds__(kThreads) void k_up2(const uint16_t *__restrict__ x, int n_coarse, int C,
                                                  uint16_t *__restrict__ y) {
    const int nf = 2 * n_coarse;
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    const long total = (long)nf * nf * nf * C;
    if (e >= total) return;
    const int c = (int)(e % C);
    const long q = e / C;
    const int k = (int)(q % nf), j = (int)((q / nf) % nf), i = (int)(q / ((long)nf * nf));
    y[e] = x[(((long)(i >> 1) * n_coarse + (j >> 1)) * n_coarse + (k >> 1)) * C + c];
}

// dz[p][c] = (sum of the 8 children of p in dy) * (mask[p][c] > 0)
__global__ __launch_bounds__(kThreads) void k_up2_bwd(const uint16_t *__restrict__ dy, int n_coarse, int C,
                                                      const uint16_t *__restrict__ mask, int mask_cs,
                                                      uint16_t *__restrict__ dz) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    const long total = (long)n_coarse * n_coarse * n_coarse * C;
    if (e >= total) return;
    const int c = (int)(e % C);
    const long p = e / C;
    const int nf = 2 * n_coarse;
    const int k = (int)(p % n_coarse), j = (int)((p / n_coarse) % n_coarse), i = (int)(p / ((long)n_coarse * n_coarse));
    float s = 0.f;
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int d = 0; d < 2; d++)
                s += bf2f(dy[(((long)(2 * i + a) * nf + (2 * j + b)) * nf + (2 * k + d)) * C + c]);
    if (!(bf2f(mask[p * mask_cs + c]) > 0.f)) s = 0.f;
    dz[e] = f2bf(s);
}

// dz[p][c] = src[p][c] * (mask[p][c] > 0) for a channel slice
__global__ __launch_bounds__(kThreads) void k_mask(const uint16_t *__restrict__ src, int src_cs, long P, int C,
                                                   const uint16_t *__restrict__ mask, int mask_cs,
                                                   uint16_t *__restrict__ dz) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= P * C) return;
    const int c = (int)(e % C);
    const long p = e / C;
    dz[e] = bf2f(mask[p * mask_cs + c]) > 0.f ? src[p * src_cs + c] : (uint16_t)0;
}

// The same three element-wise kernels on 8 channels (16 bytes) a thread, for
// channel counts and strides that are multiples of 8 on 16-byte aligned
// buffers (every use in the network): one vector load and store per thread
// instead of eight 2-byte ones.
__global__ __launch_bounds__(kThreads) void k_up2_v8(const uint16_t *__restrict__ x, int n_coarse, int C,
                                                     uint16_t *__restrict__ y) {
    const int nf = 2 * n_coarse, C8 = C >> 3;
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    const long total = (long)nf * nf * nf * C8;
    if (e >= total) return;
    const int c = (int)(e % C8) * 8;
    const long q = e / C8;
    const int k = (int)(q % nf), j = (int)((q / nf) % nf), i = (int)(q / ((long)nf * nf));
    *reinterpret_cast<v8s *>(y + q * C + c) =
        *reinterpret_cast<const v8s *>(x + (((long)(i >> 1) * n_coarse + (j >> 1)) * n_coarse + (k >> 1)) * C + c);
}

__global__ __launch_bounds__(kThreads) void k_up2_bwd_v8(const uint16_t *__restrict__ dy, int n_coarse, int C,
                                                         const uint16_t *__restrict__ mask, int mask_cs,
                                                         uint16_t *__restrict__ dz) {
    const int C8 = C >> 3, nf = 2 * n_coarse;
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    const long total = (long)n_coarse * n_coarse * n_coarse * C8;
    if (e >= total) return;
    const int c = (int)(e % C8) * 8;
    const long p = e / C8;
    const int k = (int)(p % n_coarse), j = (int)((p / n_coarse) % n_coarse), i = (int)(p / ((long)n_coarse * n_coarse));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 2; a++)
        for (int b = 0; b < 2; b++)
            for (int d = 0; d < 2; d++) {
                const v8s v = *reinterpret_cast<const v8s *>(
                    dy + (((long)(2 * i + a) * nf + (2 * j + b)) * nf + (2 * k + d)) * C + c);
#pragma unroll
                for (int u = 0; u < 8; u++) s[u] += bf2f((uint16_t)v[u]);
            }
    const v8s m = *reinterpret_cast<const v8s *>(mask + p * mask_cs + c);
    v8s o;
#pragma unroll
    for (int u = 0; u < 8; u++) o[u] = (short)(bf2f((uint16_t)m[u]) > 0.f ? f2bf(s[u]) : f2bf(0.f));
    *reinterpret_cast<v8s *>(dz + p * C + c) = o;
}

__global__ __launch_bounds__(kThreads) void k_mask_v8(const uint16_t *__restrict__ src, int src_cs, long P, int C,
                                                      const uint16_t *__restrict__ mask, int mask_cs,
                                                      uint16_t *__restrict__ dz) {
    const int C8 = C >> 3;
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= P * C8) return;
    const int c = (int)(e % C8) * 8;
    const long p = e / C8;
    const v8s v = *reinterpret_cast<const v8s *>(src + p * src_cs + c);
    const v8s m = *reinterpret_cast<const v8s *>(mask + p * mask_cs + c);
    v8s o;
#pragma unroll
    for (int u = 0; u < 8; u++) o[u] = bf2f((uint16_t)m[u]) > 0.f ? v[u] : (short)0;
    *reinterpret_cast<v8s *>(dz + p * C + c) = o;
}

// network input: [p][16] with channels (rho_T, rho_R, 0, ...)
__global__ __launch_bounds__(kThreads) void k_pack_input(const float *__restrict__ a, const float *__restrict__ b,
                                                         long P, uint16_t *__restrict__ x) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= P * 16) return;
    const int c = (int)(e & 15);
    const long p = e >> 4;
    x[e] = c == 0 ? f2bf(a[p]) : c == 1 ? f2bf(b[p]) : (uint16_t)0;
}

// the head's pre-activation gradient dz[p][16] = scale dv[c][p] for an
// arbitrary loss (channels >= 3 zero)
__global__ __launch_bounds__(kThreads) void k_pack_head_grad(const float *__restrict__ dv, long P, float scale,
                                                             uint16_t *__restrict__ dz) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= P * 16) return;
    const int c = (int)(e & 15);
    const long p = e >> 4;
    dz[e] = c < 3 ? f2bf(scale * dv[c * P + p]) : (uint16_t)0;
}

// MSE: per-block partial sums of (v - t)^2 (double) and the head's
// pre-activation gradient dz[p][16] = 2 (v - t) / numel (channels >= 3 zero)
__global__ __launch_bounds__(kThreads) void k_mse(const float *__restrict__ v, const float *__restrict__ tgt, long P,
                                                  double *__restrict__ partials, uint16_t *__restrict__ dz) {
    const long p = (long)blockIdx.x * kThreads + threadIdx.x;
    double s = 0.0;
    if (p < P) {
        const float scale = 2.f / (3.f * (float)P);
        for (int c = 0; c < 16; c++) {
            float gval = 0.f;
            if (c < 3) {
                const float r = v[c * P + p] - tgt[c * P + p];
                s += (double)r * r;
                gval = scale * r;
            }
            dz[p * 16 + c] = f2bf(gval);
        }
    }
    __shared__ double sm[kThreads];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = sm[0];
}

// *out += scale * sum(partials), one workgroup: strided per-thread sums,
// then a tree in LDS (a fixed order)
__global__ __launch_bounds__(kThreads) void k_sum(const double *__restrict__ partials, int n, double scale,
                                                  double *__restrict__ out) {
    __shared__ double sm[kThreads];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kThreads) s += partials[i];
    sm[threadIdx.x] = s;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sm[threadIdx.x] += sm[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out += scale * sm[0];
}

// Adam with bias-corrected moments, FP32
__global__ __launch_bounds__(kThreads) void k_adam(long n, float *__restrict__ w, const float *__restrict__ g,
                                                   float *__restrict__ m, float *__restrict__ s, float lr, float b1,
                                                   float b2, float eps, float c1, float c2) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const float gr = g[e];
    const float mi = b1 * m[e] + (1.f - b1) * gr;
    const float si = b2 * s[e] + (1.f - b2) * gr * gr;
    m[e] = mi;
    s[e] = si;
    w[e] -= lr * (mi / c1) / (sqrtf(si / c2) + eps);
}

// BF16 weight copies: fwd[t][co_pad][ci_pad] and bwd[t][ci_pad][co_pad] from
// the master W[co][ci][t] (zero padding)
__global__ __launch_bounds__(kThreads) void k_pack_weights(const float *__restrict__ W, int cout, int cin, int cout_pad,
                                                           int cin_pad, uint16_t *__restrict__ fwd,
                                                           uint16_t *__restrict__ bwd) {
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= 27 * cout_pad * cin_pad) return;
    const int ci = e % cin_pad, co = (e / cin_pad) % cout_pad, t = e / (cin_pad * cout_pad);
    const uint16_t v = (co < cout && ci < cin) ? f2bf(W[((long)co * cin + ci) * 27 + t]) : (uint16_t)0;
    fwd[e] = v;
    bwd[((long)t * cin_pad + ci) * cout_pad + co] = v;
}

// out[c][p] = x[p][c] for c < C (BF16 channel-last to FP32 channel-first)
__global__ __launch_bounds__(kThreads) void k_unpack(const uint16_t *__restrict__ x, int cs, int C, long P,
                                                     float *__restrict__ out) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= P * C) return;
    const long p = e % P;
    const int c = (int)(e / P);
    out[e] = bf2f(x[p * cs + c]);
}

__global__ __launch_bounds__(kThreads) void k_fill_f32(long n, float v, float *__restrict__ x) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) x[e] = v;
}

__global__ __launch_bounds__(kThreads) void k_scale_f32(long n, float s, float *__restrict__ x) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) x[e] *= s;
}

inline unsigned blocks(long n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

hipError_t launch_conv(int mode, const ConvArgs &a, hipStream_t s) {
    const long P = (long)a.n_out * a.n_out * a.n_out;
    if (P % 64 || a.cin % 16 || a.cout % 16 || a.cout > 64 || a.cin > 64 || a.in_cs % 4) return hipErrorInvalidValue;
    // four point blocks per wavefront (64 points) and every channel block on
    // grids of 32^3 and more; on the small grids one point block and one
    // channel block per wavefront, the channel blocks over gridDim.y, which
    // would otherwise leave the GPU idle
    const bool wide = P >= 32768;
    const int NB = a.cout / 16;
    if (NB != 1 && NB != 2 && NB != 4) return hipErrorInvalidValue;
    // stride-1 layers on grids of 32^3 and more: the LDS-tiled kernel (one
    // channel block per workgroup on 32^3, all of them on larger grids)
    const bool tiled_ok = (mode == CONV_FWD1 || mode == CONV_BWD1) && a.n_out % kCT3 == 0 && a.in_cs % 8 == 0 &&
                          (reinterpret_cast<uintptr_t>(a.in) & 15) == 0 && wide;
    if (tiled_ok) {
        const unsigned ntile = (unsigned)((a.n_out / kCT1) * (a.n_out / kCT2) * (a.n_out / kCT3));
        const bool split = P <= 32768;
        const dim3 grid(ntile, split ? NB : 1);
#define REGN_TILED(M)                                                                                  \
    do {                                                                                               \
        if (split || NB == 1) hipLaunchKernelGGL((k_conv_tiled<M, 1>), grid, dim3(kThreads), 0, s, a); \
        else if (NB == 2) hipLaunchKernelGGL((k_conv_tiled<M, 2>), grid, dim3(kThreads), 0, s, a);     \
        else hipLaunchKernelGGL((k_conv_tiled<M, 4>), grid, dim3(kThreads), 0, s, a);                  \
    } while (0)
        if (mode == CONV_FWD1) REGN_TILED(CONV_FWD1);
        else REGN_TILED(CONV_BWD1);
#undef REGN_TILED
        return hipGetLastError();
    }
    if (mode == CONV_BWD2 && a.n_out == 2 * a.n_in && a.n_in % 16 == 0) {
        const long waves = 8L * a.n_in * a.n_in * (a.n_in / 16);
        const dim3 g2((unsigned)((waves + 3) / 4));
        if (NB == 1) hipLaunchKernelGGL(k_conv_bwd2<1>, g2, dim3(kThreads), 0, s, a);
        else if (NB == 2) hipLaunchKernelGGL(k_conv_bwd2<2>, g2, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL(k_conv_bwd2<4>, g2, dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    // the 16^3 grid (and smaller): taps split over each workgroup's waves
    if (P <= 4096 && mode != CONV_BWD2) {
        const dim3 gk((unsigned)(P / 16), NB);
        switch (mode) {
        case CONV_FWD1: hipLaunchKernelGGL(k_conv_ksplit<CONV_FWD1>, gk, dim3(kThreads), 0, s, a); break;
        case CONV_FWD2: hipLaunchKernelGGL(k_conv_ksplit<CONV_FWD2>, gk, dim3(kThreads), 0, s, a); break;
        case CONV_BWD1: hipLaunchKernelGGL(k_conv_ksplit<CONV_BWD1>, gk, dim3(kThreads), 0, s, a); break;
        default: return hipErrorInvalidValue;
        }
        return hipGetLastError();
    }
    // a stride-2 forward onto a 32^3 grid takes the small-grid form too:
    // with 64 points per wavefront it would fill only half of the SIMDs
    const bool wide_direct = wide && !(mode == CONV_FWD2 && P <= 32768);
    const unsigned nb = (unsigned)((P / (wide_direct ? 64 : 16) + 3) / 4);
    const dim3 grid(nb, wide_direct ? 1 : NB);
#define REGN_CONV(M)                                                                                  \
    do {                                                                                              \
        if (!wide_direct) hipLaunchKernelGGL((k_conv<M, 1, 1>), grid, dim3(kThreads), 0, s, a);      \
        else if (NB == 1) hipLaunchKernelGGL((k_conv<M, 1, 4>), grid, dim3(kThreads), 0, s, a);      \
        else if (NB == 2) hipLaunchKernelGGL((k_conv<M, 2, 4>), grid, dim3(kThreads), 0, s, a);      \
        else hipLaunchKernelGGL((k_conv<M, 4, 4>), grid, dim3(kThreads), 0, s, a);                   \
    } while (0)
    switch (mode) {
    case CONV_FWD1: REGN_CONV(CONV_FWD1); break;
    case CONV_FWD2: REGN_CONV(CONV_FWD2); break;
    case CONV_BWD1: REGN_CONV(CONV_BWD1); break;
    case CONV_BWD2: REGN_CONV(CONV_BWD2); break;
    default: return hipErrorInvalidValue;
    }
#undef REGN_CONV
    return hipGetLastError();
}

int wgrad_chunks(int n_out) {
    const long P = (long)n_out * n_out * n_out;
    return (int)((P + wgrad_chunk(P) - 1) / wgrad_chunk(P));
}

hipError_t launch_wgrad(int mode, const WgradArgs &a, hipStream_t s) {
    const long P = (long)a.n_out * a.n_out * a.n_out;
    if (P % kSlice || a.cin % 16 || a.cout % 16 || a.cin > 64 || a.cout > 64 || a.x_cs % 4 || a.dz_cs % 4)
        return hipErrorInvalidValue;
    // stride-1 layers on 32^3 and finer grids: the tiled kernel (whole
    // 4x4x16 tiles, whole chunks of them, 16-byte input loads)
    if (mode == CONV_FWD1 && a.n_in == a.n_out && a.n_out >= 32 && a.n_out % kCT3 == 0 && a.x_cs % 8 == 0 &&
        wgrad_chunk(P) % kWTile == 0 && (a.cout == 16 || a.cout == 32 || a.cout == 64)) {
        const dim3 gt(wgrad_chunks(a.n_out), a.cin / 16, 3);
        if (a.cout == 16) hipLaunchKernelGGL(k_wgrad_tiled<1>, gt, dim3(kThreads), 0, s, a);
        else if (a.cout == 32) hipLaunchKernelGGL(k_wgrad_tiled<2>, gt, dim3(kThreads), 0, s, a);
        else hipLaunchKernelGGL(k_wgrad_tiled<4>, gt, dim3(kThreads), 0, s, a);
        return hipGetLastError();
    }
    const dim3 grid(wgrad_chunks(a.n_out), 27);
    if (mode == CONV_FWD1) hipLaunchKernelGGL(k_wgrad<CONV_FWD1>, grid, dim3(kThreads), 0, s, a);
    else if (mode == CONV_FWD2) hipLaunchKernelGGL(k_wgrad<CONV_FWD2>, grid, dim3(kThreads), 0, s, a);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_wgrad_reduce(const float *partials, const float *bias_partials, int chunks, int cout, int cin,
                               int cout_real, int cin_real, float scale, float *dW, float *db, hipStream_t s) {
    const long n = (long)cout_real * cin_real * 27 + cout_real;
    hipLaunchKernelGGL(k_wgrad_reduce, dim3((unsigned)((n + kRedW - 1) / kRedW)), dim3(kThreads), 0, s, partials,
                       bias_partials, chunks, cout,
                       cin, cout_real, cin_real, scale, dW, db);
    return hipGetLastError();
}

static bool al16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

hipError_t launch_up2(const uint16_t *x, int n_coarse, int C, uint16_t *y, hipStream_t s) {
    const long total = 8L * n_coarse * n_coarse * n_coarse * C;
    if (C % 8 == 0 && al16(x) && al16(y))
        hipLaunchKernelGGL(k_up2_v8, dim3(blocks(total / 8)), dim3(kThreads), 0, s, x, n_coarse, C, y);
    else
        hipLaunchKernelGGL(k_up2, dim3(blocks(total)), dim3(kThreads), 0, s, x, n_coarse, C, y);
    return hipGetLastError();
}

hipError_t launch_up2_bwd(const uint16_t *dy, int n_coarse, int C, const uint16_t *mask, int mask_cs, uint16_t *dz,
                          hipStream_t s) {
    const long total = (long)n_coarse * n_coarse * n_coarse * C;
    if (C % 8 == 0 && mask_cs % 8 == 0 && al16(dy) && al16(mask) && al16(dz))
        hipLaunchKernelGGL(k_up2_bwd_v8, dim3(blocks(total / 8)), dim3(kThreads), 0, s, dy, n_coarse, C, mask, mask_cs,
                           dz);
    else
        hipLaunchKernelGGL(k_up2_bwd, dim3(blocks(total)), dim3(kThreads), 0, s, dy, n_coarse, C, mask, mask_cs, dz);
    return hipGetLastError();
}

hipError_t launch_mask(const uint16_t *src, int src_cs, long P, int C, const uint16_t *mask, int mask_cs, uint16_t *dz,
                       hipStream_t s) {
    if (C % 8 == 0 && src_cs % 8 == 0 && mask_cs % 8 == 0 && al16(src) && al16(mask) && al16(dz))
        hipLaunchKernelGGL(k_mask_v8, dim3(blocks(P * C / 8)), dim3(kThreads), 0, s, src, src_cs, P, C, mask, mask_cs,
                           dz);
    else
        hipLaunchKernelGGL(k_mask, dim3(blocks(P * C)), dim3(kThreads), 0, s, src, src_cs, P, C, mask, mask_cs, dz);
    return hipGetLastError();
}

hipError_t launch_pack_input(const float *a, const float *b, long P, uint16_t *x, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_input, dim3(blocks(P * 16)), dim3(kThreads), 0, s, a, b, P, x);
    return hipGetLastError();
}

int mse_blocks(long P) { return (int)blocks(P); }

hipError_t launch_pack_head_grad(const float *dv, long P, float scale, uint16_t *dz, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_head_grad, dim3(blocks(P * 16)), dim3(kThreads), 0, s, dv, P, scale, dz);
    return hipGetLastError();
}

hipError_t launch_mse(const float *v, const float *tgt, long P, double *partials, double *loss_acc, double scale,
                      uint16_t *dz, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(blocks(P)), dim3(kThreads), 0, s, v, tgt, P, partials, dz);
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(kThreads), 0, s, partials, (int)blocks(P), scale, loss_acc);
    return hipGetLastError();
}

hipError_t launch_adam(long n, float *w, const float *g, float *m, float *v, float lr, float b1, float b2, float eps,
                       int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(blocks(n)), dim3(kThreads), 0, s, n, w, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_pack_weights(const float *W, int cout, int cin, int cout_pad, int cin_pad, uint16_t *fwd,
                               uint16_t *bwd, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_weights, dim3(blocks(27L * cout_pad * cin_pad)), dim3(kThreads), 0, s, W, cout, cin,
                       cout_pad, cin_pad, fwd, bwd);
    return hipGetLastError();
}

hipError_t launch_unpack(const uint16_t *x, int cs, int C, long P, float *out, hipStream_t s) {
    hipLaunchKernelGGL(k_unpack, dim3(blocks(P * C)), dim3(kThreads), 0, s, x, cs, C, P, out);
    return hipGetLastError();
}

hipError_t launch_fill_f32(long n, float v, float *x, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_f32, dim3(blocks(n)), dim3(kThreads), 0, s, n, v, x);
    return hipGetLastError();
}

hipError_t launch_scale_f32(long n, float sc, float *x, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_f32, dim3(blocks(n)), dim3(kThreads), 0, s, n, sc, x);
    return hipGetLastError();
}

}  // namespace regn
