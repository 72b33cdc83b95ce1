// Spectral kernels for gfx950 (section III-B1 of the paper: Fourier
// discretisation on the periodic grid; section III-C1: derivatives need only
// 1D FFTs along the differentiated axis, while P, lap^2 and lap^-2 are
// diagonal after a full 3D transform).
//
// Line FFTs of any length 2^a 3^b 5^c up to 1024 run in LDS: a workgroup
// stages L complex lines of one axis as a [j][l] tile (pitch >= L), runs a
// Stockham autosort FFT with radix-8/4/2/3/5 passes between two LDS buffers,
// and writes the tile back. 256-point lines (two radix-16 passes) keep each
// thread's 16 elements in registers instead, with one LDS exchange between
// the passes, reading and writing HBM directly in the 3D transforms. For
// the x1 and x2 axes the L lines are L adjacent x3 columns, so every global
// access is a coalesced row of L complex values; for the contiguous x3 axis
// the lines are loaded along x3 and transposed into the tile. Real data is
// packed two lines per complex line: a derivative symbol i k~ is Hermitian,
// so the real and imaginary parts of the inverse are the two derivatives;
// the R2C/C2R passes split and merge the two half spectra explicitly.
#include "common.hpp"

namespace regk {

bool make_plan(int n, FftPlan *p) {
    p->n = n;
    p->npass = 0;
    int m = n;
    while (m % 8 == 0 && p->npass < 12) {
        p->radix[p->npass++] = 8;
        m /= 8;
    }
    while (m % 4 == 0 && p->npass < 12) {
        p->radix[p->npass++] = 4;
        m /= 4;
    }
    while (m % 2 == 0 && p->npass < 12) {
        p->radix[p->npass++] = 2;
        m /= 2;
    }
    while (m % 3 == 0 && p->npass < 12) {
        p->radix[p->npass++] = 3;
        m /= 3;
    }
    while (m % 5 == 0 && p->npass < 12) {
        p->radix[p->npass++] = 5;
        m /= 5;
    }
    return m == 1;
}

namespace {

constexpr int kThreads = 256;

// Workgroups are dispatched round-robin over the 8 XCDs (one L2 each). The
// strided line transforms below read and write 64-byte pieces of 128-byte
// lines, the other half belonging to the neighbouring block along x3; this
// index keeps neighbouring blocks on one XCD (XCD x takes the x-th
// contiguous share of gridDim.x), so the line is fetched into one L2 once.
__device__ __forceinline__ int xcd_local_block() {
    const unsigned b = blockIdx.x, nb = gridDim.x;
    const unsigned q = nb / 8, r = nb % 8;
    const unsigned x = b % 8, t = b / 8;
    const unsigned base = x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q;
    return (int)(base + t);
}

// row pitch of a tile of L lines in LDS; padded tiles (transposed loads) add
// one element per row against bank conflicts
__host__ __device__ inline int tile_pitch(int L, bool padded) { return (padded && L > 1) ? L + 1 : L; }

template <typename C>
__device__ __forceinline__ C cmul(C a, C b) {
    C r;
    r.x = a.x * b.x - a.y * b.y;
    r.y = a.x * b.y + a.y * b.x;
    return r;
}
template <typename C>
__device__ __forceinline__ C cadd(C a, C b) {
    C r;
    r.x = a.x + b.x;
    r.y = a.y + b.y;
    return r;
}
template <typename C>
__device__ __forceinline__ C csub(C a, C b) {
    C r;
    r.x = a.x - b.x;
    r.y = a.y - b.y;
    return r;
}
// multiply by sign*i
template <typename C>
__device__ __forceinline__ C cmul_si(C a, int sign) {
    C r;
    r.x = sign > 0 ? -a.y : a.y;
    r.y = sign > 0 ? a.x : -a.x;
    return r;
}

// R-point DFT with kernel exp(sign 2 pi i r q / R), R in {2, 3, 4, 5, 8}
template <typename T, int R>
__device__ __forceinline__ void butterfly(cplx_t<T> *v, int sign) {
    using C = cplx_t<T>;
    if (R == 8) {
        // even and odd samples through 4-point DFTs, then X_k = E_k + w^k O_k
        // and X_{k+4} = E_k - w^k O_k with w = exp(sign 2 pi i / 8) =
        // h (1 + sign i), w^2 = sign i, w^3 = h (-1 + sign i), h = sqrt(2)/2
        C e[4] = {v[0], v[2], v[4], v[6]}, o[4] = {v[1], v[3], v[5], v[7]};
        butterfly<T, 4>(e, sign);
        butterfly<T, 4>(o, sign);
        const T h = T(0.70710678118654752440084436210485);
        C t1 = cadd(o[1], cmul_si(o[1], sign));
        t1.x *= h;
        t1.y *= h;
        const C t2 = cmul_si(o[2], sign);
        C t3 = csub(cmul_si(o[3], sign), o[3]);
        t3.x *= h;
        t3.y *= h;
        v[0] = cadd(e[0], o[0]);
        v[4] = csub(e[0], o[0]);
        v[1] = cadd(e[1], t1);
        v[5] = csub(e[1], t1);
        v[2] = cadd(e[2], t2);
        v[6] = csub(e[2], t2);
        v[3] = cadd(e[3], t3);
        v[7] = csub(e[3], t3);
    } else if (R == 4) {
        const C s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
        const C s13 = cadd(v[1], v[3]), d13 = cmul_si(csub(v[1], v[3]), sign);
        v[0] = cadd(s02, s13);
        v[2] = csub(s02, s13);
        v[1] = cadd(d02, d13);
        v[3] = csub(d02, d13);
    } else if (R == 2) {
        const C a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    } else if (R == 5) {
        // with t1 = v1 + v4, t2 = v2 + v3, t3 = v1 - v4, t4 = v2 - v3:
        // X0 = v0 + t1 + t2; X1, X4 = a1 +- b1; X2, X3 = a2 +- b2 with
        // a1 = v0 + c1 t1 + c2 t2, a2 = v0 + c2 t1 + c1 t2,
        // b1 = sign i (s1 t3 + s2 t4), b2 = sign i (s2 t3 - s1 t4),
        // c_m = cos(2 pi m / 5), s_m = sin(2 pi m / 5)
        const T c1 = T(0.30901699437494742410229341718282), c2 = T(-0.80901699437494742410229341718282);
        const T s1 = T(0.95105651629515357211643933337938), s2 = T(0.58778525229247312916870595463907);
        const C t1 = cadd(v[1], v[4]), t2 = cadd(v[2], v[3]), t3 = csub(v[1], v[4]), t4 = csub(v[2], v[3]);
        C a1, a2, e1, e2;
        a1.x = v[0].x + c1 * t1.x + c2 * t2.x;
        a1.y = v[0].y + c1 * t1.y + c2 * t2.y;
        a2.x = v[0].x + c2 * t1.x + c1 * t2.x;
        a2.y = v[0].y + c2 * t1.y + c1 * t2.y;
        e1.x = s1 * t3.x + s2 * t4.x;
        e1.y = s1 * t3.y + s2 * t4.y;
        e2.x = s2 * t3.x - s1 * t4.x;
        e2.y = s2 * t3.y - s1 * t4.y;
        const C b1 = cmul_si(e1, sign), b2 = cmul_si(e2, sign);
        v[0] = cadd(v[0], cadd(t1, t2));
        v[1] = cadd(a1, b1);
        v[4] = csub(a1, b1);
        v[2] = cadd(a2, b2);
        v[3] = csub(a2, b2);
    } else {  // R == 3
        const T h = T(0.86602540378443864676372317075294);  // sqrt(3)/2
        const C s = cadd(v[1], v[2]), d = csub(v[1], v[2]);
        C m;
        m.x = v[0].x - T(0.5) * s.x;
        m.y = v[0].y - T(0.5) * s.y;
        C e = cmul_si(d, sign);
        e.x *= h;
        e.y *= h;
        v[0] = cadd(v[0], s);
        v[1] = cadd(m, e);
        v[2] = csub(m, e);
    }
}

// One radix-R Stockham pass over L = 2^lgL lines, element (j, l) at
// a[j*pitch + l]: combines R sub-transforms of length Ns into one of length
// Ns*R. tw[m] = exp(-2 pi i m / n) (in LDS); the inverse conjugates.
template <typename T, int R>
__device__ __forceinline__ void fft_pass(const cplx_t<T> *a, cplx_t<T> *b, int n, int Ns, int lgL, int pitch,
                                         int sign, const cplx_t<T> *tw) {
    using C = cplx_t<T>;
    const int L = 1 << lgL;
    const int nr = n / R;
    const int tstep = n / (Ns * R);
    const bool pow2 = (Ns & (Ns - 1)) == 0;
    for (int e = threadIdx.x; e < nr * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        int k, q;
        if (pow2) {
            k = j & (Ns - 1);
            q = j - k;
        } else {
            q = (j / Ns) * Ns;
            k = j - q;
        }
        C v[R];
#pragma unroll
        for (int r = 0; r < R; r++) v[r] = a[(j + r * nr) * pitch + l];
#pragma unroll
        for (int r = 1; r < R; r++) {
            C w = tw[r * k * tstep];
            if (sign > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        butterfly<T, R>(v, sign);
        const int d = q * R + k;
#pragma unroll
        for (int r = 0; r < R; r++) b[(d + r * Ns) * pitch + l] = v[r];
    }
}

// 16-point DFT with kernel exp(sign 2 pi i r q / 16) in registers, natural
// order in and out: x[4 n1 + n2] -> X[k1 + 4 k2] as 4-point DFTs over n1,
// twiddles exp(sign 2 pi i n2 k1 / 16), 4-point DFTs over n2.
template <typename T>
__device__ __forceinline__ void dft16(cplx_t<T> x[16], int sign) {
    using C = cplx_t<T>;
    // cos and sin of 2 pi m / 16, m = 0..9
    const T c16[10] = {T(1), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                       T(0), T(-0.38268343236508977173), T(-0.70710678118654752440), T(-0.92387953251128675613),
                       T(-1), T(-0.92387953251128675613)};
    const T s16[10] = {T(0), T(0.38268343236508977173), T(0.70710678118654752440), T(0.92387953251128675613),
                       T(1), T(0.92387953251128675613), T(0.70710678118654752440), T(0.38268343236508977173),
                       T(0), T(-0.38268343236508977173)};
    C y[4][4];
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) {
        C v[4] = {x[n2], x[4 + n2], x[8 + n2], x[12 + n2]};
        butterfly<T, 4>(v, sign);
#pragma unroll
        for (int k1 = 0; k1 < 4; k1++) y[n2][k1] = v[k1];
    }
#pragma unroll
    for (int n2 = 1; n2 < 4; n2++)
#pragma unroll
        for (int k1 = 1; k1 < 4; k1++) {
            C w;
            w.x = c16[n2 * k1];
            w.y = sign > 0 ? s16[n2 * k1] : -s16[n2 * k1];
            y[n2][k1] = cmul(y[n2][k1], w);
        }
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        C v[4] = {y[0][k1], y[1][k1], y[2][k1], y[3][k1]};
        butterfly<T, 4>(v, sign);
#pragma unroll
        for (int k2 = 0; k2 < 4; k2++) x[k1 + 4 * k2] = v[k2];
    }
}

// 256-point Stockham FFT of 2^lgL lines as two radix-16 passes, each
// thread transforming 16 elements of one line in registers (fewer passes,
// index computations and twiddle reads than four radix-4 passes); result in
// a, ends with a barrier.
template <typename T>
__device__ cplx_t<T> *fft256_r16(cplx_t<T> *a, cplx_t<T> *b, int lgL, int pitch, int sign, const cplx_t<T> *tw) {
    using C = cplx_t<T>;
    const int L = 1 << lgL;
    // Ns = 1: b[16 j + r] = DFT16(a[j + 16 r])
    for (int e = threadIdx.x; e < 16 * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        C v[16];
#pragma unroll
        for (int r = 0; r < 16; r++) v[r] = a[(j + 16 * r) * pitch + l];
        dft16<T>(v, sign);
#pragma unroll
        for (int r = 0; r < 16; r++) b[(16 * j + r) * pitch + l] = v[r];
    }
    __syncthreads();
    // Ns = 16: a[j + 16 r] = DFT16(b[j + 16 r] w^(r j)), w = exp(sign 2 pi i / 256)
    for (int e = threadIdx.x; e < 16 * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        C v[16];
#pragma unroll
        for (int r = 0; r < 16; r++) v[r] = b[(j + 16 * r) * pitch + l];
#pragma unroll
        for (int r = 1; r < 16; r++) {
            C w = tw[r * j];
            if (sign > 0) w.y = -w.y;
            v[r] = cmul(v[r], w);
        }
        dft16<T>(v, sign);
#pragma unroll
        for (int r = 0; r < 16; r++) a[(j + 16 * r) * pitch + l] = v[r];
    }
    __syncthreads();
    return a;
}

// Stockham FFT of 2^lgL lines held in LDS; returns the buffer that holds the
// result (natural order); ends with a barrier.
template <typename T>
__device__ cplx_t<T> *lds_fft(cplx_t<T> *a, cplx_t<T> *b, const FftPlan &pl, int lgL, int pitch, int sign,
                              const cplx_t<T> *tw) {
    using C = cplx_t<T>;
    if (pl.n == 256) return fft256_r16<T>(a, b, lgL, pitch, sign, tw);
    int Ns = 1;
    for (int ps = 0; ps < pl.npass; ps++) {
        const int R = pl.radix[ps];
        if (R == 8) fft_pass<T, 8>(a, b, pl.n, Ns, lgL, pitch, sign, tw);
        else if (R == 4) fft_pass<T, 4>(a, b, pl.n, Ns, lgL, pitch, sign, tw);
        else if (R == 2) fft_pass<T, 2>(a, b, pl.n, Ns, lgL, pitch, sign, tw);
        else if (R == 3) fft_pass<T, 3>(a, b, pl.n, Ns, lgL, pitch, sign, tw);
        else fft_pass<T, 5>(a, b, pl.n, Ns, lgL, pitch, sign, tw);
        __syncthreads();
        C *t = a;
        a = b;
        b = t;
        Ns *= R;
    }
    return a;
}

template <typename T>
__device__ __forceinline__ void stage_twiddles(cplx_t<T> *twl, const cplx_t<T> *__restrict__ tw, int n) {
    for (int m = threadIdx.x; m < n; m += blockDim.x) twl[m] = tw[m];
}

// wavenumber of index m on an axis of length n, and its odd variant (Nyquist -> 0)
__device__ __forceinline__ int kwave(int m, int n) { return 2 * m <= n ? m : m - n; }
__device__ __forceinline__ int kwave_odd(int m, int n) { return 2 * m == n ? 0 : kwave(m, n); }

// multiply row j of the tile by the derivative symbol i k~_j / n
template <typename T>
__device__ __forceinline__ void deriv_symbol(cplx_t<T> *R, int n, int lgL, int pitch) {
    using C = cplx_t<T>;
    const int L = 1 << lgL;
    const T inv = T(1) / T(n);
    for (int e = threadIdx.x; e < n * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        const T f = T(kwave_odd(j, n)) * inv;
        const C z = R[j * pitch + l];
        C w;
        w.x = -f * z.y;
        w.y = f * z.x;
        R[j * pitch + l] = w;
    }
}

// ----------------------------------------------------------- derivatives

// Lines along axis 0 or 1 of a real field: the tile holds L complex columns,
// each the pair of adjacent x3 columns (2l, 2l+1) of the block.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_deriv_strided(Grid g, FftPlan pl, const cplx_t<T> *__restrict__ tw,
                                                            int axis, const T *__restrict__ u, long in_stride,
                                                            T *__restrict__ out, long out_stride, int accumulate,
                                                            int lgL) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = 1 << lgL;
    const int n = pl.n;
    C *A = reinterpret_cast<C *>(smem);
    C *B = A + n * L;
    C *twl = B + n * L;
    const int ncol = g.n3 / 2;
    const int nb3 = (ncol + L - 1) >> lgL;
    const int blk = xcd_local_block();
    const int outer = blk / nb3, cb = blk - outer * nb3;
    const int leff = min(L, ncol - cb * L);
    long base, stride;
    if (axis == 1) {
        base = (long)outer * g.n2 * g.n3 + 2L * cb * L;
        stride = g.n3;
    } else {
        base = (long)outer * g.n3 + 2L * cb * L;
        stride = (long)g.n2 * g.n3;
    }
    const T *src = u + blockIdx.y * in_stride;
    T *dst = out + blockIdx.y * out_stride;
    stage_twiddles<T>(twl, tw, n);
    for (int e = threadIdx.x; e < n * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        C z;
        z.x = T(0);
        z.y = T(0);
        if (l < leff) z = *reinterpret_cast<const C *>(src + base + j * stride + 2 * l);
        A[j * L + l] = z;
    }
    __syncthreads();
    C *R = lds_fft<T>(A, B, pl, lgL, L, -1, twl);
    deriv_symbol<T>(R, n, lgL, L);
    __syncthreads();
    C *Q = lds_fft<T>(R, R == A ? B : A, pl, lgL, L, +1, twl);
    for (int e = threadIdx.x; e < n * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        if (l >= leff) continue;
        C *p = reinterpret_cast<C *>(dst + base + j * stride + 2 * l);
        C z = Q[j * L + l];
        if (accumulate) {
            const C o = *p;
            z.x += o.x;
            z.y += o.y;
        }
        *p = z;
    }
}

// Lines along the contiguous x3 axis: L complex lines, each the pair of real
// lines (r0 + 2l, r0 + 2l + 1) with r = i1*n2 + i2; each wavefront moves
// whole lines, lanes along x3.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_deriv_x3(Grid g, FftPlan pl, const cplx_t<T> *__restrict__ tw,
                                                       const T *__restrict__ u, long in_stride, T *__restrict__ out,
                                                       long out_stride, int accumulate, int lgL) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = 1 << lgL, pitch = tile_pitch(L, true);
    const int n = pl.n;  // == n3
    C *A = reinterpret_cast<C *>(smem);
    C *B = A + n * pitch;
    C *twl = B + n * pitch;
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    const T *src = u + blockIdx.y * in_stride;
    T *dst = out + blockIdx.y * out_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    stage_twiddles<T>(twl, tw, n);
    for (int l = wave; l < L; l += nw)
        for (int j = lane; j < n; j += 64) {
            C z;
            z.x = T(0);
            z.y = T(0);
            if (l < leff) {
                z.x = src[(r0 + 2 * l) * n + j];
                z.y = src[(r0 + 2 * l + 1) * n + j];
            }
            A[j * pitch + l] = z;
        }
    __syncthreads();
    C *R = lds_fft<T>(A, B, pl, lgL, pitch, -1, twl);
    deriv_symbol<T>(R, n, lgL, pitch);
    __syncthreads();
    C *Q = lds_fft<T>(R, R == A ? B : A, pl, lgL, pitch, +1, twl);
    for (int l = wave; l < leff; l += nw)
        for (int j = lane; j < n; j += 64) {
            const C z = Q[j * pitch + l];
            T *p0 = dst + (r0 + 2 * l) * n + j;
            T *p1 = dst + (r0 + 2 * l + 1) * n + j;
            if (accumulate) {
                *p0 += z.x;
                *p1 += z.y;
            } else {
                *p0 = z.x;
                *p1 = z.y;
            }
        }
}

// ------------------------------------------------------------ 3D transforms

// R2C along x3 of a pair of real lines per complex line, then split the two
// half spectra: X_a = (Z_k + conj Z_{n-k})/2, X_b = (Z_k - conj Z_{n-k})/(2i).
template <typename Tr, typename T>
__global__ __launch_bounds__(kThreads) void k_r2c_x3(Grid g, FftPlan pl, const cplx_t<T> *__restrict__ tw,
                                                     const Tr *__restrict__ x, long in_stride, cplx_t<T> *__restrict__ H,
                                                     long h_stride, int lgL) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = 1 << lgL, pitch = tile_pitch(L, true);
    const int n = pl.n, nh = n / 2 + 1;
    C *A = reinterpret_cast<C *>(smem);
    C *B = A + n * pitch;
    C *twl = B + n * pitch;
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    const Tr *src = x + blockIdx.y * in_stride;
    C *dst = H + blockIdx.y * h_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    stage_twiddles<T>(twl, tw, n);
    for (int l = wave; l < L; l += nw)
        for (int j = lane; j < n; j += 64) {
            C z;
            z.x = T(0);
            z.y = T(0);
            if (l < leff) {
                z.x = T(src[(r0 + 2 * l) * n + j]);
                z.y = T(src[(r0 + 2 * l + 1) * n + j]);
            }
            A[j * pitch + l] = z;
        }
    __syncthreads();
    C *R = lds_fft<T>(A, B, pl, lgL, pitch, -1, twl);
    for (int l = wave; l < leff; l += nw)
        for (int k = lane; k < nh; k += 64) {
            const C z = R[k * pitch + l];
            const C zc = R[(k == 0 ? 0 : n - k) * pitch + l];
            C xa, xb;
            xa.x = T(0.5) * (z.x + zc.x);
            xa.y = T(0.5) * (z.y - zc.y);
            xb.x = T(0.5) * (z.y + zc.y);
            xb.y = T(-0.5) * (z.x - zc.x);
            dst[(r0 + 2 * l) * nh + k] = xa;
            dst[(r0 + 2 * l + 1) * nh + k] = xb;
        }
}

// 256-point x3 transforms of 2^LG complex lines (pairs of real lines) per
// workgroup, 16 threads per line, each holding elements j + 16 r (r = 0..15)
// of its line in registers; the exchange between the two radix-16 passes goes
// through LDS (line-major, rows skewed by one element per 16 against bank
// conflicts).
constexpr int kX3Pitch = 256 + 16;

// Exchange step and second radix-16 pass shared by both x3 kernels: v holds
// the first pass's output DFT16(a[j + 16 r]) of this thread's line; on return
// v[r] = X[j + 16 r].
template <typename T>
__device__ __forceinline__ void x3_second_pass(cplx_t<T> v[16], cplx_t<T> *line_buf, int j, const cplx_t<T> *twl,
                                               int sign) {
    using C = cplx_t<T>;
#pragma unroll
    for (int r = 0; r < 16; r++) line_buf[17 * j + r] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = line_buf[j + 17 * r];
#pragma unroll
    for (int r = 1; r < 16; r++) {
        C w = twl[r * j];
        if (sign > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
    }
    dft16<T>(v, sign);
}

// R2C along x3 (n3 = 256) of line pairs, then the split of the two half
// spectra as in k_r2c_x3; Z_{n-k} comes from lane 16 - j of the same line.
template <typename Tr, typename T, int LG>
__global__ __launch_bounds__(16 << LG) void k_r2c256_x3(Grid g, const cplx_t<T> *__restrict__ tw,
                                                        const Tr *__restrict__ x, long in_stride,
                                                        cplx_t<T> *__restrict__ H, long h_stride) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG, n = 256, nh = 129;
    __shared__ C buf[L * kX3Pitch];
    __shared__ C twl[256];
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    for (int m = threadIdx.x; m < n; m += 16 << LG) twl[m] = tw[m];
    const int j = threadIdx.x & 15, l = threadIdx.x >> 4;
    const bool live = l < leff;
    const Tr *sa = x + blockIdx.y * in_stride + (r0 + 2 * l) * n;
    const Tr *sb = sa + n;
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        v[r].x = T(0);
        v[r].y = T(0);
        if (live) {
            v[r].x = T(sa[j + 16 * r]);
            v[r].y = T(sb[j + 16 * r]);
        }
    }
    dft16<T>(v, -1);
    x3_second_pass<T>(v, buf + l * kX3Pitch, j, twl, -1);
    const int lane = threadIdx.x & 63, partner = (lane & ~15) | ((16 - j) & 15);
    C *da = H + blockIdx.y * h_stride + (r0 + 2 * l) * nh;
    C *db = da + nh;
#pragma unroll
    for (int r = 0; r <= 8; r++) {
        // lane 16 - j holds Z_{n-k} for k = j + 16 r in v[15 - r]; lane 0
        // holds its own in v[(16 - r) mod 16]
        const C give = j == 0 ? v[(16 - r) & 15] : v[15 - r];
        C zc;
        zc.x = __shfl(give.x, partner, 64);
        zc.y = __shfl(give.y, partner, 64);
        const C z = v[r];
        const int k = j + 16 * r;
        if (live && k < nh) {
            C xa, xb;
            xa.x = T(0.5) * (z.x + zc.x);
            xa.y = T(0.5) * (z.y - zc.y);
            xb.x = T(0.5) * (z.y + zc.y);
            xb.y = T(-0.5) * (z.x - zc.x);
            da[k] = xa;
            db[k] = xb;
        }
    }
}

// C2R along x3 (n3 = 256): merge two half spectra into Z = X_a + i X_b as in
// k_c2r_x3, inverse FFT, scale, real part to line r0 + 2 l, imaginary part to
// line r0 + 2 l + 1.
template <typename T, typename Tr, int LG>
__global__ __launch_bounds__(16 << LG) void k_c2r256_x3(Grid g, const cplx_t<T> *__restrict__ tw,
                                                        const cplx_t<T> *__restrict__ H, long h_stride,
                                                        Tr *__restrict__ out, long out_stride, T scale) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG, n = 256, nh = 129;
    __shared__ C buf[L * kX3Pitch];
    __shared__ C twl[256];
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    for (int m = threadIdx.x; m < n; m += 16 << LG) twl[m] = tw[m];
    const int j = threadIdx.x & 15, l = threadIdx.x >> 4;
    const bool live = l < leff;
    const C *sa = H + blockIdx.y * h_stride + (r0 + 2 * l) * nh;
    const C *sb = sa + nh;
    // each half-spectrum value is loaded once, k = j + 16 r for r < 8 and
    // k = n/2 by lane 0; Z_k for k > n/2 needs X_{n-k}, which lane 16 - j
    // loaded as its r' = 15 - r (lane 0: its own r' = 16 - r)
    C da[9], db[9];
#pragma unroll
    for (int r = 0; r < 9; r++) {
        da[r].x = T(0);
        da[r].y = T(0);
        db[r] = da[r];
        if (live && (r < 8 || j == 0)) {
            da[r] = sa[j + 16 * r];
            db[r] = sb[j + 16 * r];
        }
    }
    if (j == 0) {  // k = 0 and k = n/2 are real
        da[0].y = T(0);
        db[0].y = T(0);
        da[8].y = T(0);
        db[8].y = T(0);
    }
    const int lane = threadIdx.x & 63, partner = (lane & ~15) | ((16 - j) & 15);
    C v[16];
#pragma unroll
    for (int r = 0; r < 8; r++) {
        v[r].x = da[r].x - db[r].y;
        v[r].y = da[r].y + db[r].x;
    }
#pragma unroll
    for (int r = 8; r < 16; r++) {
        // selects on values (a select of the two array elements would be
        // lowered through private memory)
        const bool own = j == 0;
        const C a0 = da[16 - r], a1 = da[15 - r], b0 = db[16 - r], b1 = db[15 - r];
        C xa, xb;
        xa.x = __shfl(own ? a0.x : a1.x, partner, 64);
        xa.y = __shfl(own ? a0.y : a1.y, partner, 64);
        xb.x = __shfl(own ? b0.x : b1.x, partner, 64);
        xb.y = __shfl(own ? b0.y : b1.y, partner, 64);
        if (r == 8 && j == 0) {  // k = n/2 itself
            v[r].x = xa.x - xb.y;
            v[r].y = xa.y + xb.x;
        } else {
            v[r].x = xa.x + xb.y;
            v[r].y = xb.x - xa.y;
        }
    }
    dft16<T>(v, +1);
    x3_second_pass<T>(v, buf + l * kX3Pitch, j, twl, +1);
    if (live) {
        Tr *oa = out + blockIdx.y * out_stride + (r0 + 2 * l) * n;
        Tr *ob = oa + n;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            oa[j + 16 * r] = Tr(scale * v[r].x);
            ob[j + 16 * r] = Tr(scale * v[r].y);
        }
    }
}

// In-place complex FFT of the half spectrum along axis 0 or 1.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_c2c_strided(Grid g, FftPlan pl, const cplx_t<T> *__restrict__ tw,
                                                          int axis, cplx_t<T> *__restrict__ H, long h_stride, int sign,
                                                          int lgL) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = 1 << lgL;
    const int n = pl.n;
    C *A = reinterpret_cast<C *>(smem);
    C *B = A + n * L;
    C *twl = B + n * L;
    const int nh = g.n3h();
    const int nb3 = (nh + L - 1) >> lgL;
    const int blk = xcd_local_block();
    const int outer = blk / nb3, cb = blk - outer * nb3;
    const int leff = min(L, nh - cb * L);
    long base, stride;
    if (axis == 1) {
        base = (long)outer * g.n2 * nh + (long)cb * L;
        stride = nh;
    } else {
        base = (long)outer * nh + (long)cb * L;
        stride = (long)g.n2 * nh;
    }
    C *h = H + blockIdx.y * h_stride;
    stage_twiddles<T>(twl, tw, n);
    for (int e = threadIdx.x; e < n * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        C z;
        z.x = T(0);
        z.y = T(0);
        if (l < leff) z = h[base + j * stride + l];
        A[j * L + l] = z;
    }
    __syncthreads();
    C *R = lds_fft<T>(A, B, pl, lgL, L, sign, twl);
    for (int e = threadIdx.x; e < n * L; e += blockDim.x) {
        const int l = e & (L - 1), j = e >> lgL;
        if (l < leff) h[base + j * stride + l] = R[j * L + l];
    }
}

// Spectral derivative of 256-point lines in registers: the thread that ends
// the forward transform with X[j + 16 r] (r = 0..15) multiplies by the
// symbol i k~ / n and starts the inverse transform with exactly those
// values, so forward and inverse need one LDS exchange each.
template <typename T>
__device__ __forceinline__ void deriv256_symbol(cplx_t<T> v[16], int j) {
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const T f = T(kwave_odd(j + 16 * r, 256)) * T(1.0 / 256.0);
        const T x = v[r].x;
        v[r].x = -f * v[r].y;
        v[r].y = f * x;
    }
}

// Along x3 (n3 = 256): 2^LG line pairs per workgroup, 16 threads per pair,
// the real lines r0 + 2 l and r0 + 2 l + 1 packed as one complex line (the
// derivative is real, so it acts on both parts separately).
template <typename T, int LG>
__global__ __launch_bounds__(16 << LG) void k_deriv256_x3(Grid g, const cplx_t<T> *__restrict__ tw,
                                                          const T *__restrict__ u, long in_stride,
                                                          T *__restrict__ out, long out_stride, int accumulate) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG, n = 256;
    __shared__ C buf[L * kX3Pitch];
    __shared__ C twl[256];
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    for (int m = threadIdx.x; m < n; m += 16 << LG) twl[m] = tw[m];
    const int j = threadIdx.x & 15, l = threadIdx.x >> 4;
    const bool live = l < leff;
    const T *sa = u + blockIdx.y * in_stride + (r0 + 2 * l) * n;
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        v[r].x = T(0);
        v[r].y = T(0);
        if (live) {
            v[r].x = sa[j + 16 * r];
            v[r].y = sa[n + j + 16 * r];
        }
    }
    C *line_buf = buf + l * kX3Pitch;
    dft16<T>(v, -1);
    x3_second_pass<T>(v, line_buf, j, twl, -1);
    deriv256_symbol<T>(v, j);
    dft16<T>(v, +1);
    __syncthreads();  // every thread has read the forward exchange
    x3_second_pass<T>(v, line_buf, j, twl, +1);
    if (live) {
        T *oa = out + blockIdx.y * out_stride + (r0 + 2 * l) * n;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            T *pa = oa + j + 16 * r, *pb = pa + n;
            if (accumulate) {
                *pa += v[r].x;
                *pb += v[r].y;
            } else {
                *pa = v[r].x;
                *pb = v[r].y;
            }
        }
    }
}

// Exchange and second radix-16 pass of a 256-point column transform with
// 2^LG columns per workgroup (rows skewed by one element per 16 in LDS);
// v holds DFT16(a[j + 16 r]) on entry and X[j + 16 r] on return.
template <typename T, int LG>
__device__ __forceinline__ void col_second_pass(cplx_t<T> v[16], cplx_t<T> *buf, int j, int l,
                                                const cplx_t<T> *twl, int sign) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG;
#pragma unroll
    for (int r = 0; r < 16; r++) buf[(16 * j + r) * L + j + l] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = buf[(j + 16 * r) * L + r + l];
#pragma unroll
    for (int r = 1; r < 16; r++) {
        C w = twl[r * j];
        if (sign > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
    }
    dft16<T>(v, sign);
}

// Along x1 or x2 (that axis 256 long) of real fields: 2^LG complex columns
// per workgroup, each the pair of adjacent x3 columns (2 c, 2 c + 1).
template <typename T, int LG>
__global__ __launch_bounds__(16 << LG) void k_deriv256_strided(Grid g, const cplx_t<T> *__restrict__ tw, int axis,
                                                               const T *__restrict__ u, long in_stride,
                                                               T *__restrict__ out, long out_stride, int accumulate) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG;
    __shared__ C buf[256 * L + 16];
    __shared__ C twl[256];
    const int ncol = g.n3 / 2;
    const int nb3 = (ncol + L - 1) >> LG;
    const int blk = xcd_local_block();
    const int outer = blk / nb3, cb = blk - outer * nb3;
    const int leff = min(L, ncol - cb * L);
    long base, stride;
    if (axis == 1) {
        base = (long)outer * g.n2 * g.n3 + 2L * cb * L;
        stride = g.n3;
    } else {
        base = (long)outer * g.n3 + 2L * cb * L;
        stride = (long)g.n2 * g.n3;
    }
    for (int m = threadIdx.x; m < 256; m += 16 << LG) twl[m] = tw[m];
    const int l = threadIdx.x & (L - 1), j = threadIdx.x >> LG;
    const bool live = l < leff;
    const T *src = u + blockIdx.y * in_stride + base + 2 * l;
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        v[r].x = T(0);
        v[r].y = T(0);
        if (live) v[r] = *reinterpret_cast<const C *>(src + (long)(j + 16 * r) * stride);
    }
    dft16<T>(v, -1);
    col_second_pass<T, LG>(v, buf, j, l, twl, -1);
    deriv256_symbol<T>(v, j);
    dft16<T>(v, +1);
    __syncthreads();  // every thread has read the forward exchange
    col_second_pass<T, LG>(v, buf, j, l, twl, +1);
    if (live) {
        T *dst = out + blockIdx.y * out_stride + base + 2 * l;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            C *p = reinterpret_cast<C *>(dst + (long)(j + 16 * r) * stride);
            C z = v[r];
            if (accumulate) {
                const C o = *p;
                z.x += o.x;
                z.y += o.y;
            }
            *p = z;
        }
    }
}

// 256-point complex FFT of the half spectrum along axis 0 or 1 (in place, or
// from src into H), 2^LG columns per workgroup and 16 threads per column. Each thread keeps 16
// elements of its column in registers: the first radix-16 pass reads them
// straight from HBM (rows j + 16 r), the second writes them straight back, and
// only the exchange between the passes goes through LDS (one buffer, rows
// skewed by one element per 16 against bank conflicts). Same two passes as
// fft256_r16.
template <typename T, int LG>
__global__ __launch_bounds__(16 << LG) void k_c2c256_strided(Grid g, const cplx_t<T> *__restrict__ tw, int axis,
                                                             const cplx_t<T> *src, cplx_t<T> *H, long h_stride,
                                                             int sign) {
    using C = cplx_t<T>;
    constexpr int L = 1 << LG, kRow = L, kSkew = 1;
    __shared__ C buf[256 * kRow + 16 * kSkew];
    __shared__ C twl[256];
    const int nh = g.n3h();
    const int nb3 = (nh + L - 1) >> LG;
    const int blk = xcd_local_block();
    const int outer = blk / nb3, cb = blk - outer * nb3;
    const int leff = min(L, nh - cb * L);
    long base, stride;
    if (axis == 1) {
        base = (long)outer * g.n2 * nh + (long)cb * L;
        stride = nh;
    } else {
        base = (long)outer * nh + (long)cb * L;
        stride = (long)g.n2 * nh;
    }
    C *h = H + blockIdx.y * h_stride;
    const C *hs = src + blockIdx.y * h_stride;  // == h in place
    for (int m = threadIdx.x; m < 256; m += 16 << LG) twl[m] = tw[m];
    const int l = threadIdx.x & (L - 1), j = threadIdx.x >> LG;
    const bool live = l < leff;
    C v[16];
#pragma unroll
    for (int r = 0; r < 16; r++) {
        v[r].x = T(0);
        v[r].y = T(0);
        if (live) v[r] = hs[base + (long)(j + 16 * r) * stride + l];
    }
    dft16<T>(v, sign);
    // row m = 16 j + r of the exchange buffer sits at m * kRow + (m >> 4) * kSkew
#pragma unroll
    for (int r = 0; r < 16; r++) buf[(16 * j + r) * kRow + j * kSkew + l] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; r++) v[r] = buf[(j + 16 * r) * kRow + r * kSkew + l];
#pragma unroll
    for (int r = 1; r < 16; r++) {
        C w = twl[r * j];
        if (sign > 0) w.y = -w.y;
        v[r] = cmul(v[r], w);
    }
    dft16<T>(v, sign);
    if (live) {
#pragma unroll
        for (int r = 0; r < 16; r++) h[base + (long)(j + 16 * r) * stride + l] = v[r];
    }
}

// Merge two half spectra into one complex line Z = X_a + i X_b (Hermitian
// extension for k > n/2, real parts only at k = 0 and n/2), inverse FFT,
// scale, and store the real part to line r0+2l and the imaginary part to
// line r0+2l+1.
template <typename T, typename Tr>
__global__ __launch_bounds__(kThreads) void k_c2r_x3(Grid g, FftPlan pl, const cplx_t<T> *__restrict__ tw,
                                                     const cplx_t<T> *__restrict__ H, long h_stride,
                                                     Tr *__restrict__ out, long out_stride, T scale, int lgL) {
    using C = cplx_t<T>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = 1 << lgL, pitch = tile_pitch(L, true);
    const int n = pl.n, nh = n / 2 + 1;
    C *A = reinterpret_cast<C *>(smem);
    C *B = A + n * pitch;
    C *twl = B + n * pitch;
    const long nlines = (long)g.n1 * g.n2;
    const long r0 = (long)blockIdx.x * 2 * L;
    const int leff = (int)min((long)L, (nlines - r0) / 2);
    const C *src = H + blockIdx.y * h_stride;
    Tr *dst = out + blockIdx.y * out_stride;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
    stage_twiddles<T>(twl, tw, n);
    for (int l = wave; l < L; l += nw)
        for (int j = lane; j < n; j += 64) {
            C z;
            z.x = T(0);
            z.y = T(0);
            if (l < leff) {
                if (2 * j <= n) {
                    C xa = src[(r0 + 2 * l) * nh + j], xb = src[(r0 + 2 * l + 1) * nh + j];
                    if (j == 0 || 2 * j == n) {
                        xa.y = T(0);
                        xb.y = T(0);
                    }
                    z.x = xa.x - xb.y;
                    z.y = xa.y + xb.x;
                } else {
                    const C xa = src[(r0 + 2 * l) * nh + (n - j)], xb = src[(r0 + 2 * l + 1) * nh + (n - j)];
                    z.x = xa.x + xb.y;
                    z.y = xb.x - xa.y;
                }
            }
            A[j * pitch + l] = z;
        }
    __syncthreads();
    C *R = lds_fft<T>(A, B, pl, lgL, pitch, +1, twl);
    for (int l = wave; l < leff; l += nw)
        for (int j = lane; j < n; j += 64) {
            const C z = R[j * pitch + l];
            dst[(r0 + 2 * l) * n + j] = Tr(scale * z.x);
            dst[(r0 + 2 * l + 1) * n + j] = Tr(scale * z.y);
        }
}

// Pointwise symbols on the half spectrum [n1][n2][n3/2+1].
template <typename T>
__global__ __launch_bounds__(kThreads) void k_symbol(Grid g, cplx_t<T> *__restrict__ H, long h_stride, int op, T a,
                                                     int ncomp, int leray) {
    using C = cplx_t<T>;
    const long q = (long)blockIdx.x * kThreads + threadIdx.x;
    const long Nh = g.Nh();
    if (q >= Nh) return;
    const int nh = g.n3h();
    const int m3 = (int)(q % nh);
    const long r = q / nh;
    const int m2 = (int)(r % g.n2), m1 = (int)(r / g.n2);
    const T k1 = T(kwave(m1, g.n1)), k2 = T(kwave(m2, g.n2)), k3 = T(m3);
    const T kk = k1 * k1 + k2 * k2 + k3 * k3;
    const T t1 = T(kwave_odd(m1, g.n1)), t2 = T(kwave_odd(m2, g.n2)), t3 = T(2 * m3 == g.n3 ? 0 : m3);
    const T tt = t1 * t1 + t2 * t2 + t3 * t3;
    if (op == SYM_BIHARM || op == SYM_INVBIHARM || op == SYM_GAUSS || op == SYM_PRECOND) {
        T f;
        if (op == SYM_BIHARM) f = a * kk * kk;
        else if (op == SYM_GAUSS) f = exp(T(-0.5) * a * a * kk);
        else f = kk == T(0) ? T(1) : T(1) / (a * kk * kk);
        for (int c = 0; c < ncomp; c++) {
            C z = H[c * h_stride + q];
            z.x *= f;
            z.y *= f;
            H[c * h_stride + q] = z;
        }
        if (op != SYM_PRECOND || !leray) return;
    }
    if (op == SYM_ASSEMBLE) {
        // H_c <- a |k|^4 H_c + [P] H_{3+c}
        C y0 = H[3 * h_stride + q], y1 = H[4 * h_stride + q], y2 = H[5 * h_stride + q];
        if (leray && tt > T(0)) {
            const T ir = T(1) / tt;
            const T dx = (t1 * y0.x + t2 * y1.x + t3 * y2.x) * ir, dy = (t1 * y0.y + t2 * y1.y + t3 * y2.y) * ir;
            y0.x -= t1 * dx;
            y0.y -= t1 * dy;
            y1.x -= t2 * dx;
            y1.y -= t2 * dy;
            y2.x -= t3 * dx;
            y2.y -= t3 * dy;
        }
        const T f = a * kk * kk;
        C x0 = H[q], x1 = H[h_stride + q], x2 = H[2 * h_stride + q];
        x0.x = f * x0.x + y0.x;
        x0.y = f * x0.y + y0.y;
        x1.x = f * x1.x + y1.x;
        x1.y = f * x1.y + y1.y;
        x2.x = f * x2.x + y2.x;
        x2.y = f * x2.y + y2.y;
        H[q] = x0;
        H[h_stride + q] = x1;
        H[2 * h_stride + q] = x2;
        return;
    }
    // Leray projection of components 0..2
    if (tt == T(0)) return;
    C y0 = H[q], y1 = H[h_stride + q], y2 = H[2 * h_stride + q];
    const T ir = T(1) / tt;
    const T dx = (t1 * y0.x + t2 * y1.x + t3 * y2.x) * ir, dy = (t1 * y0.y + t2 * y1.y + t3 * y2.y) * ir;
    y0.x -= t1 * dx;
    y0.y -= t1 * dy;
    y1.x -= t2 * dx;
    y1.y -= t2 * dy;
    y2.x -= t3 * dx;
    y2.y -= t3 * dy;
    H[q] = y0;
    H[h_stride + q] = y1;
    H[2 * h_stride + q] = y2;
}

// Per-block partial sums of sum_c sum_k w(k3) |k|^4 |H_c(k)|^2 with
// w = 1 on the k3 = 0 and k3 = n3/2 planes and 2 elsewhere (the half spectrum
// stands for both k and -k), accumulated in double.
// log2 of the lines per tile: the largest power of two L such that the two
// LDS buffers of n*pitch complex values plus the n twiddles fit in 64 KiB;
// padded tiles use pitch L + 1 (pitch 1 for a single line).
template <typename T>
int pick_lg_lines(int n, int cap, bool padded) {
    const long per_buffer = (65536 / (long)sizeof(cplx_t<T>) - n) / 2;
    int lg = 0;
    while (lg < 6 && (1 << (lg + 1)) <= cap && (long)n * tile_pitch(1 << (lg + 1), padded) <= per_buffer) lg++;
    return lg;
}

template <typename T>
size_t tile_lds(int n, int lg, bool padded) {
    return (2 * (size_t)n * tile_pitch(1 << lg, padded) + n) * sizeof(cplx_t<T>);
}

}  // namespace

// ---------------------------------------------------------------- launchers

template <typename T> constexpr int tw_index() { return sizeof(T) == 8 ? 1 : 0; }

template <typename T>
hipError_t spec_deriv(const SpecCtx &c, int axis, const T *u, long in_stride, T *out, long out_stride, int accumulate,
                      int ncomp, hipStream_t s) {
    using C = cplx_t<T>;
    const Grid &g = c.g;
    const FftPlan &pl = c.plan[axis];
    const C *tw = reinterpret_cast<const C *>(c.tw[tw_index<T>()][axis]);
    if (pl.n == 256) {
        constexpr int lg_max = sizeof(T) == 4 ? 4 : 3;
        if (axis == 2) {
            const long L2 = 2L << lg_max;
            const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
            hipLaunchKernelGGL((k_deriv256_x3<T, lg_max>), dim3(nb, ncomp), dim3(16 << lg_max), 0, s, g, tw, u,
                               in_stride, out, out_stride, accumulate);
            return hipGetLastError();
        }
        // columns per workgroup: 16 in FP32 (8 in FP64), fewer for narrow x3
        const int ncol = g.n3 / 2;
        int lg = 2;
        while (lg < lg_max && (1 << lg) < ncol) lg++;
        const int nb3 = (ncol + (1 << lg) - 1) >> lg;
        const unsigned nb = (unsigned)((axis == 1 ? g.n1 : g.n2) * nb3);
        if (lg == 2)
            hipLaunchKernelGGL((k_deriv256_strided<T, 2>), dim3(nb, ncomp), dim3(64), 0, s, g, tw, axis, u, in_stride,
                               out, out_stride, accumulate);
        else if (lg == 3)
            hipLaunchKernelGGL((k_deriv256_strided<T, 3>), dim3(nb, ncomp), dim3(128), 0, s, g, tw, axis, u,
                               in_stride, out, out_stride, accumulate);
        else
            hipLaunchKernelGGL((k_deriv256_strided<T, lg_max>), dim3(nb, ncomp), dim3(16 << lg_max), 0, s, g, tw,
                               axis, u, in_stride, out, out_stride, accumulate);
        return hipGetLastError();
    }
    if (axis == 2) {
        const int lg = pick_lg_lines<T>(g.n3, (int)(((long)g.n1 * g.n2) / 2), true);
        const long L2 = 2L << lg;
        const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
        hipLaunchKernelGGL(k_deriv_x3<T>, dim3(nb, ncomp), dim3(kThreads), tile_lds<T>(pl.n, lg, true), s, g, pl, tw,
                           u, in_stride, out, out_stride, accumulate, lg);
    } else {
        const int ncol = g.n3 / 2;
        const int lg = pick_lg_lines<T>(pl.n, ncol, false);
        const int nb3 = (ncol + (1 << lg) - 1) >> lg;
        const unsigned nb = (unsigned)((axis == 1 ? g.n1 : g.n2) * nb3);
        hipLaunchKernelGGL(k_deriv_strided<T>, dim3(nb, ncomp), dim3(kThreads), tile_lds<T>(pl.n, lg, false), s, g,
                           pl, tw, axis, u, in_stride, out, out_stride, accumulate, lg);
    }
    return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_cplx_copy(long n, const cplx_t<T> *__restrict__ a,
                                                        cplx_t<T> *__restrict__ b) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e < n) b[e] = a[e];
}

// the first pass reads src0 (nullptr: H itself)
template <typename T>
static void c2c_passes(const SpecCtx &c, cplx_t<T> *H, int ncomp, int sign, hipStream_t s,
                       const cplx_t<T> *src0 = nullptr) {
    using C = cplx_t<T>;
    const Grid &g = c.g;
    const int nh = g.n3h();
    for (int k = 0; k < 2; k++) {
        const int axis = sign < 0 ? 1 - k : k;  // forward: x2 then x1; inverse: x1 then x2
        const C *src = (k == 0 && src0) ? src0 : H;
        if (src != H && c.plan[axis].n != 256) {
            const long n = (long)ncomp * g.Nh();
            hipLaunchKernelGGL(k_cplx_copy<T>, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n,
                               src, H);
            src = H;
        }
        if (c.plan[axis].n == 256) {
            // 16 columns per workgroup in FP32, 8 in FP64 (32 KiB of LDS),
            // fewer when the half spectrum is narrower
            const int lg_max = sizeof(T) == 4 ? 4 : 3;
            int lg = 2;
            while (lg < lg_max && (1 << lg) < nh) lg++;
            const int nb3 = (nh + (1 << lg) - 1) >> lg;
            const unsigned nb = (unsigned)((axis == 1 ? g.n1 : g.n2) * nb3);
            const C *tw = reinterpret_cast<const C *>(c.tw[tw_index<T>()][axis]);
            if (lg == 2)
                hipLaunchKernelGGL((k_c2c256_strided<T, 2>), dim3(nb, ncomp), dim3(64), 0, s, g, tw, axis, src, H,
                                   g.Nh(), sign);
            else if (lg == 3)
                hipLaunchKernelGGL((k_c2c256_strided<T, 3>), dim3(nb, ncomp), dim3(128), 0, s, g, tw, axis, src, H,
                                   g.Nh(), sign);
            else
                hipLaunchKernelGGL((k_c2c256_strided<T, sizeof(T) == 4 ? 4 : 3>), dim3(nb, ncomp),
                                   dim3(sizeof(T) == 4 ? 256 : 128), 0, s, g, tw, axis, src, H, g.Nh(), sign);
            continue;
        }
        const int lg = pick_lg_lines<T>(c.plan[axis].n, nh, false);
        const int nb3 = (nh + (1 << lg) - 1) >> lg;
        const unsigned nb = (unsigned)((axis == 1 ? g.n1 : g.n2) * nb3);
        hipLaunchKernelGGL(k_c2c_strided<T>, dim3(nb, ncomp), dim3(kThreads), tile_lds<T>(c.plan[axis].n, lg, false),
                           s, g, c.plan[axis], reinterpret_cast<const C *>(c.tw[tw_index<T>()][axis]), axis, H,
                           g.Nh(), sign, lg);
    }
}

template <typename Tr, typename T>
hipError_t spec_forward_to(const SpecCtx &c, const Tr *x, int ncomp, void *Hout, hipStream_t s) {
    using C = cplx_t<T>;
    const Grid &g = c.g;
    C *H = reinterpret_cast<C *>(Hout);
    const C *tw = reinterpret_cast<const C *>(c.tw[tw_index<T>()][2]);
    if (g.n3 == 256) {
        constexpr int LG = sizeof(T) == 4 ? 4 : 3;
        const long L2 = 2L << LG;
        const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
        hipLaunchKernelGGL((k_r2c256_x3<Tr, T, LG>), dim3(nb, ncomp), dim3(16 << LG), 0, s, g, tw, x, g.N(), H,
                           g.Nh());
    } else {
        const int lg = pick_lg_lines<T>(g.n3, (int)(((long)g.n1 * g.n2) / 2), true);
        const long L2 = 2L << lg;
        const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
        hipLaunchKernelGGL((k_r2c_x3<Tr, T>), dim3(nb, ncomp), dim3(kThreads), tile_lds<T>(g.n3, lg, true), s, g,
                           c.plan[2], tw, x, g.N(), H, g.Nh(), lg);
    }
    c2c_passes<T>(c, H, ncomp, -1, s);
    return hipGetLastError();
}

template <typename Tr, typename T>
hipError_t spec_forward(const SpecCtx &c, const Tr *x, int ncomp, int h0, hipStream_t s) {
    return spec_forward_to<Tr, T>(c, x, ncomp, reinterpret_cast<cplx_t<T> *>(c.H) + (long)h0 * c.g.Nh(), s);
}

template <typename T, typename Tr>
hipError_t spec_inverse_from(const SpecCtx &c, void *Hin, Tr *out, int ncomp, hipStream_t s, const void *src) {
    using C = cplx_t<T>;
    const Grid &g = c.g;
    C *H = reinterpret_cast<C *>(Hin);
    c2c_passes<T>(c, H, ncomp, +1, s, reinterpret_cast<const C *>(src));
    const C *tw = reinterpret_cast<const C *>(c.tw[tw_index<T>()][2]);
    if (g.n3 == 256) {
        constexpr int LG = sizeof(T) == 4 ? 4 : 3;
        const long L2 = 2L << LG;
        const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
        hipLaunchKernelGGL((k_c2r256_x3<T, Tr, LG>), dim3(nb, ncomp), dim3(16 << LG), 0, s, g, tw, H, g.Nh(), out,
                           g.N(), T(1.0 / (double)g.N()));
        return hipGetLastError();
    }
    const int lg = pick_lg_lines<T>(g.n3, (int)(((long)g.n1 * g.n2) / 2), true);
    const long L2 = 2L << lg;
    const unsigned nb = (unsigned)(((long)g.n1 * g.n2 + L2 - 1) / L2);
    hipLaunchKernelGGL((k_c2r_x3<T, Tr>), dim3(nb, ncomp), dim3(kThreads), tile_lds<T>(g.n3, lg, true), s, g,
                       c.plan[2], tw, H, g.Nh(), out, g.N(), T(1.0 / (double)g.N()), lg);
    return hipGetLastError();
}

template <typename T, typename Tr>
hipError_t spec_inverse(const SpecCtx &c, Tr *out, int ncomp, hipStream_t s) {
    return spec_inverse_from<T, Tr>(c, c.H, out, ncomp, s, nullptr);
}

template <typename T>
hipError_t spec_symbol(const SpecCtx &c, int op, double a, int ncomp, int leray, hipStream_t s) {
    using C = cplx_t<T>;
    const Grid &g = c.g;
    const unsigned nb = (unsigned)((g.Nh() + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_symbol<T>, dim3(nb), dim3(kThreads), 0, s, g, reinterpret_cast<C *>(c.H), g.Nh(), op, T(a),
                       ncomp, leray);
    return hipGetLastError();
}

// ------------------------------------------------ spectral velocity vectors
// Velocity-space vectors kept on the half spectrum: three components of
// [n1][n2][n3/2+1] complex double values, the unnormalised forward transform
// of the real field. Inner products follow Parseval,
// <u, w> = h1 h2 h3 / N sum_k u^(k) conj(w^(k)), with the half spectrum
// weighted 1 on the k3 = 0 and k3 = n3/2 planes and 2 elsewhere.

// H (complex T, components 0..2) = v^ (complex double)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vec_load(long n, const double2 *__restrict__ v,
                                                       cplx_t<T> *__restrict__ H) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const double2 z = v[e];
    cplx_t<T> o;
    o.x = T(z.x);
    o.y = T(z.y);
    H[e] = o;
}

// Pointwise operators on spectral velocity vectors:
//  VEC_ASSEMBLE: out = a |k|^4 x + [P] y     (y complex T, promoted)
//  VEC_PRECOND:  out = x / (a |k|^4) (x at k = 0), then [P]
//  VEC_LERAY:    out = P x
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vec_symbol(Grid g, int op, const double2 *__restrict__ x,
                                                         const cplx_t<T> *__restrict__ y, double a, int leray,
                                                         double2 *__restrict__ out) {
    const long q = (long)blockIdx.x * kThreads + threadIdx.x;
    const long Nh = g.Nh();
    if (q >= Nh) return;
    const int nh = g.n3h();
    const int m3 = (int)(q % nh);
    const long r = q / nh;
    const int m2 = (int)(r % g.n2), m1 = (int)(r / g.n2);
    const double k1 = kwave(m1, g.n1), k2 = kwave(m2, g.n2), k3 = m3;
    const double kk = k1 * k1 + k2 * k2 + k3 * k3;
    const double t1 = kwave_odd(m1, g.n1), t2 = kwave_odd(m2, g.n2), t3 = (2 * m3 == g.n3 ? 0 : m3);
    const double tt = t1 * t1 + t2 * t2 + t3 * t3;
    double2 v[3];
    if (op == VEC_ASSEMBLE) {
        for (int c = 0; c < 3; c++) {
            const cplx_t<T> z = y[c * Nh + q];
            v[c] = make_double2((double)z.x, (double)z.y);
        }
    } else {
        for (int c = 0; c < 3; c++) v[c] = x[c * Nh + q];
        if (op == VEC_PRECOND && kk > 0.0) {
            const double f = 1.0 / (a * kk * kk);
            for (int c = 0; c < 3; c++) {
                v[c].x *= f;
                v[c].y *= f;
            }
        }
    }
    if ((leray || op == VEC_LERAY) && tt > 0.0) {
        const double ir = 1.0 / tt;
        const double dx = (t1 * v[0].x + t2 * v[1].x + t3 * v[2].x) * ir;
        const double dy = (t1 * v[0].y + t2 * v[1].y + t3 * v[2].y) * ir;
        v[0].x -= t1 * dx;
        v[0].y -= t1 * dy;
        v[1].x -= t2 * dx;
        v[1].y -= t2 * dy;
        v[2].x -= t3 * dx;
        v[2].y -= t3 * dy;
    }
    if (op == VEC_ASSEMBLE) {
        const double f = a * kk * kk;
        for (int c = 0; c < 3; c++) {
            const double2 z = x[c * Nh + q];
            v[c].x = f * z.x + v[c].x;
            v[c].y = f * z.y + v[c].y;
        }
    }
    for (int c = 0; c < 3; c++) out[c * Nh + q] = v[c];
}

// Per-block partial sums of sum_c sum_k w(k3) Re(a_c conj(b_c)) (mode 0) or
// sum_c sum_k w(k3) |k|^4 |a_c|^2 (mode 1), in a fixed order.
template <typename B>
__global__ __launch_bounds__(kThreads) void k_vec_dot(Grid g, int mode, const double2 *__restrict__ a,
                                                      const B *__restrict__ b, double *__restrict__ partials) {
    const long Nh = g.Nh();
    const int nh = g.n3h();
    double acc = 0.0;
    for (long q = (long)blockIdx.x * kThreads + threadIdx.x; q < Nh; q += (long)gridDim.x * kThreads) {
        const int m3 = (int)(q % nh);
        const double w = (m3 == 0 || 2 * m3 == g.n3) ? 1.0 : 2.0;
        double s = 0.0;
        if (mode == 0) {
            for (int c = 0; c < 3; c++) {
                const double2 x = a[c * Nh + q];
                const B y = b[c * Nh + q];
                s += x.x * (double)y.x + x.y * (double)y.y;
            }
        } else {
            const long r = q / nh;
            const int m2 = (int)(r % g.n2), m1 = (int)(r / g.n2);
            const double k1 = kwave(m1, g.n1), k2 = kwave(m2, g.n2), k3 = m3;
            const double kk = k1 * k1 + k2 * k2 + k3 * k3;
            for (int c = 0; c < 3; c++) {
                const double2 x = a[c * Nh + q];
                s += x.x * x.x + x.y * x.y;
            }
            s *= kk * kk;
        }
        acc += w * s;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    __shared__ double ws[kThreads / 64];
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < kThreads / 64; i++) t += ws[i];
        partials[blockIdx.x] = t;
    }
}

// ---------------------------------------------- fused Krylov vector passes
// Reductions below write one partial per block of a grid-stride loop over the
// half spectrum; k_finalize adds them in a fixed order.

__device__ __forceinline__ void block_sum2(double &x, double &y, double *__restrict__ px,
                                           double *__restrict__ py) {
    for (int off = 32; off > 0; off >>= 1) {
        x += __shfl_down(x, off, 64);
        y += __shfl_down(y, off, 64);
    }
    __shared__ double wsx[kThreads / 64], wsy[kThreads / 64];
    if ((threadIdx.x & 63) == 0) {
        wsx[threadIdx.x >> 6] = x;
        wsy[threadIdx.x >> 6] = y;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tx = 0.0, ty = 0.0;
        for (int i = 0; i < kThreads / 64; i++) {
            tx += wsx[i];
            ty += wsy[i];
        }
        if (px) px[blockIdx.x] = tx;
        if (py) py[blockIdx.x] = ty;
    }
}

struct ModeInfo {
    double kk, t1, t2, t3, tt, w;
};

__device__ __forceinline__ ModeInfo mode_info(const Grid &g, long q) {
    const int nh = g.n3h();
    const int m3 = (int)(q % nh);
    const long r = q / nh;
    const int m2 = (int)(r % g.n2), m1 = (int)(r / g.n2);
    ModeInfo mi;
    const double k1 = kwave(m1, g.n1), k2 = kwave(m2, g.n2), k3 = m3;
    mi.kk = k1 * k1 + k2 * k2 + k3 * k3;
    mi.t1 = kwave_odd(m1, g.n1);
    mi.t2 = kwave_odd(m2, g.n2);
    mi.t3 = (2 * m3 == g.n3 ? 0 : m3);
    mi.tt = mi.t1 * mi.t1 + mi.t2 * mi.t2 + mi.t3 * mi.t3;
    mi.w = (m3 == 0 || 2 * m3 == g.n3) ? 1.0 : 2.0;
    return mi;
}

__device__ __forceinline__ void leray3(const ModeInfo &mi, double2 v[3]) {
    if (mi.tt > 0.0) {
        const double ir = 1.0 / mi.tt;
        const double dx = (mi.t1 * v[0].x + mi.t2 * v[1].x + mi.t3 * v[2].x) * ir;
        const double dy = (mi.t1 * v[0].y + mi.t2 * v[1].y + mi.t3 * v[2].y) * ir;
        v[0].x -= mi.t1 * dx;
        v[0].y -= mi.t1 * dy;
        v[1].x -= mi.t2 * dx;
        v[1].y -= mi.t2 * dy;
        v[2].x -= mi.t3 * dx;
        v[2].y -= mi.t3 * dy;
    }
}

// z = M r: inverse biharmonic (identity at k = 0), then P when leray
__device__ __forceinline__ void precond3(const ModeInfo &mi, double beta, int leray, const double2 r[3],
                                         double2 z[3]) {
    const double f = mi.kk > 0.0 ? 1.0 / (beta * mi.kk * mi.kk) : 1.0;
    for (int c = 0; c < 3; c++) z[c] = make_double2(f * r[c].x, f * r[c].y);
    if (leray) leray3(mi, z);
}

// The Krylov vectors s, r, p of the PCG are stored as complex T (double
// with double fields, float with float fields: the matvec sees p rounded to
// T in either case); every update is computed in double from the stored
// values and rounded once when stored.
template <typename T>
__device__ __forceinline__ double2 ld2(const cplx_t<T> &z) {
    return make_double2((double)z.x, (double)z.y);
}
// streaming load (non-temporal: the Krylov passes read each value once)
template <typename T>
__device__ __forceinline__ double2 ld2nt(const cplx_t<T> *ptr) {
    typedef T v2 __attribute__((ext_vector_type(2)));
    const v2 z = __builtin_nontemporal_load(reinterpret_cast<const v2 *>(ptr));
    return make_double2((double)z.x, (double)z.y);
}
__device__ __forceinline__ double2 ldv_nt(const cplx_t<float> *ptr) { return ld2nt<float>(ptr); }
__device__ __forceinline__ double2 ldv_nt(const double2 *ptr) {
    return ld2nt<double>(reinterpret_cast<const cplx_t<double> *>(ptr));
}
template <typename T>
__device__ __forceinline__ cplx_t<T> st2(double2 z) {
    cplx_t<T> o;
    o.x = T(z.x);
    o.y = T(z.y);
    return o;
}

// PCG set-up of a Newton step: s = 0, r = -g, p = M r (also into H);
// partials of <r, M r>
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pcg_start(Grid g, const double2 *__restrict__ gv, double beta, int leray,
                                                        cplx_t<T> *__restrict__ s, cplx_t<T> *__restrict__ r,
                                                        cplx_t<T> *__restrict__ p, double *__restrict__ part_rz) {
    const long Nh = g.Nh();
    double rz = 0.0, dummy = 0.0;
    for (long q = (long)blockIdx.x * kThreads + threadIdx.x; q < Nh; q += (long)gridDim.x * kThreads) {
        const ModeInfo mi = mode_info(g, q);
        double2 rv[3], zv[3];
        for (int c = 0; c < 3; c++) {
            const double2 x = gv[c * Nh + q];
            rv[c] = ld2<T>(st2<T>(make_double2(-x.x, -x.y)));
        }
        precond3(mi, beta, leray, rv, zv);
        double acc = 0.0;
        for (int c = 0; c < 3; c++) {
            s[c * Nh + q] = st2<T>(make_double2(0.0, 0.0));
            r[c * Nh + q] = st2<T>(rv[c]);
            p[c * Nh + q] = st2<T>(zv[c]);
            acc += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
        }
        rz += mi.w * acc;
    }
    block_sum2(rz, dummy, part_rz, nullptr);
}

// PCG step: q = beta |k|^4 p + [P] y recomputed from the matvec's
// transformed b~ (bit for bit the q of its curvature), s += a p, r -= a q;
// partials of <r, r> and <r, M r>
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pcg_step(Grid g, double a, const cplx_t<T> *__restrict__ p,
                                                       const cplx_t<T> *__restrict__ y, double beta, int leray,
                                                       cplx_t<T> *__restrict__ s, cplx_t<T> *__restrict__ r,
                                                       double *__restrict__ part_rr, double *__restrict__ part_rz) {
    const long Nh = g.Nh();
    double rr = 0.0, rz = 0.0;
    for (long q = (long)blockIdx.x * kThreads + threadIdx.x; q < Nh; q += (long)gridDim.x * kThreads) {
        const ModeInfo mi = mode_info(g, q);
        double2 qv[3], rv[3], zv[3];
        for (int c = 0; c < 3; c++) qv[c] = ld2nt<T>(y + c * Nh + q);
        if (leray) leray3(mi, qv);
        const double f = beta * mi.kk * mi.kk;
        for (int c = 0; c < 3; c++) {
            const double2 pc = ld2nt<T>(p + c * Nh + q);
            qv[c].x = f * pc.x + qv[c].x;
            qv[c].y = f * pc.y + qv[c].y;
            double2 sc = ld2nt<T>(s + c * Nh + q), rc = ld2nt<T>(r + c * Nh + q);
            sc.x += a * pc.x;
            sc.y += a * pc.y;
            rc.x -= a * qv[c].x;
            rc.y -= a * qv[c].y;
            s[c * Nh + q] = st2<T>(sc);
            const cplx_t<T> rs = st2<T>(rc);
            r[c * Nh + q] = rs;
            rv[c] = ld2<T>(rs);
        }
        precond3(mi, beta, leray, rv, zv);
        double arr = 0.0, arz = 0.0;
        for (int c = 0; c < 3; c++) {
            arr += rv[c].x * rv[c].x + rv[c].y * rv[c].y;
            arz += rv[c].x * zv[c].x + rv[c].y * zv[c].y;
        }
        rr += mi.w * arr;
        rz += mi.w * arz;
    }
    block_sum2(rr, rz, part_rr, part_rz);
}

// next direction p = M r + b p
template <typename T>
__global__ __launch_bounds__(kThreads) void k_pcg_direction(Grid g, const cplx_t<T> *__restrict__ r, double b,
                                                            double beta, int leray, cplx_t<T> *__restrict__ p) {
    const long Nh = g.Nh();
    const long q = (long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= Nh) return;
    const ModeInfo mi = mode_info(g, q);
    double2 rv[3], zv[3];
    for (int c = 0; c < 3; c++) rv[c] = ld2nt<T>(r + c * Nh + q);
    precond3(mi, beta, leray, rv, zv);
    for (int c = 0; c < 3; c++) {
        const double2 pc = ld2nt<T>(p + c * Nh + q);
        double2 o;
        o.x = zv[c].x + b * pc.x;
        o.y = zv[c].y + b * pc.y;
        p[c * Nh + q] = st2<T>(o);
    }
}

// out = x + a y for a velocity vector x (complex double) and a Krylov vector
// y (complex T)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_vec_axpy_krylov(long n, const double2 *__restrict__ x, double a,
                                                              const cplx_t<T> *__restrict__ y,
                                                              double2 *__restrict__ out) {
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const double2 xv = x[e], yv = ld2<T>(y[e]);
    out[e] = make_double2(xv.x + a * yv.x, xv.y + a * yv.y);
}

// out = a |k|^4 x + [P] y (y complex T) with partials of <x, out> (dot 1) or
// <out, out> (dot 2)
template <typename T, typename X>
__global__ __launch_bounds__(kThreads) void k_vec_assemble_dot(Grid g, const X *__restrict__ x,
                                                               const cplx_t<T> *__restrict__ y, double a, int leray,
                                                               int dot, double2 *__restrict__ out,
                                                               double *__restrict__ part) {
    const long Nh = g.Nh();
    double acc = 0.0, dummy = 0.0;
    for (long q = (long)blockIdx.x * kThreads + threadIdx.x; q < Nh; q += (long)gridDim.x * kThreads) {
        const ModeInfo mi = mode_info(g, q);
        double2 v[3];
        for (int c = 0; c < 3; c++) v[c] = ld2nt<T>(y + c * Nh + q);
        if (leray) leray3(mi, v);
        const double f = a * mi.kk * mi.kk;
        double loc = 0.0;
        for (int c = 0; c < 3; c++) {
            const double2 xc = ldv_nt(x + c * Nh + q);
            v[c].x = f * xc.x + v[c].x;
            v[c].y = f * xc.y + v[c].y;
            if (out) out[c * Nh + q] = v[c];
            loc += dot == 1 ? xc.x * v[c].x + xc.y * v[c].y : v[c].x * v[c].x + v[c].y * v[c].y;
        }
        acc += mi.w * loc;
    }
    block_sum2(acc, dummy, part, nullptr);
}

// Spectral resampling between grids: destination mode (q1, q2, q3) takes the
// source mode of the same wavenumber, scaled by Nd/Ns, when |k_j| <
// min(ns_j, nd_j)/2 on every axis (the Nyquist planes of the smaller grid are
// dropped), and 0 otherwise.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_resample(Grid gs, Grid gd, const cplx_t<T> *__restrict__ Hs,
                                                       cplx_t<T> *__restrict__ Hd, int ncomp, T scale) {
    using C = cplx_t<T>;
    const long q = (long)blockIdx.x * kThreads + threadIdx.x;
    if (q >= gd.Nh()) return;
    const int nhd = gd.n3h(), nhs = gs.n3h();
    const int q3 = (int)(q % nhd);
    const long r = q / nhd;
    const int q2 = (int)(r % gd.n2), q1 = (int)(r / gd.n2);
    const int k1 = kwave(q1, gd.n1), k2 = kwave(q2, gd.n2), k3 = q3;
    const bool keep = 2 * abs(k1) < min(gs.n1, gd.n1) && 2 * abs(k2) < min(gs.n2, gd.n2) &&
                      2 * k3 < min(gs.n3, gd.n3);
    long src = 0;
    if (keep) {
        const int s1 = k1 < 0 ? k1 + gs.n1 : k1, s2 = k2 < 0 ? k2 + gs.n2 : k2;
        src = ((long)s1 * gs.n2 + s2) * nhs + k3;
    }
    for (int c = 0; c < ncomp; c++) {
        C z;
        z.x = T(0);
        z.y = T(0);
        if (keep) {
            z = Hs[c * gs.Nh() + src];
            z.x *= scale;
            z.y *= scale;
        }
        Hd[c * gd.Nh() + q] = z;
    }
}

template <typename T>
hipError_t spec_resample(const SpecCtx &src, const SpecCtx &dst, int ncomp, hipStream_t s) {
    using C = cplx_t<T>;
    const unsigned nb = (unsigned)((dst.g.Nh() + kThreads - 1) / kThreads);
    const T scale = T((double)dst.g.N() / (double)src.g.N());
    hipLaunchKernelGGL(k_resample<T>, dim3(nb), dim3(kThreads), 0, s, src.g, dst.g,
                       reinterpret_cast<const C *>(src.H), reinterpret_cast<C *>(dst.H), ncomp, scale);
    return hipGetLastError();
}

template <typename T>
hipError_t vec_load(const SpecCtx &c, const double *vhat, void *H, hipStream_t s) {
    const long n = 3 * c.g.Nh();
    hipLaunchKernelGGL(k_vec_load<T>, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n,
                       reinterpret_cast<const double2 *>(vhat), reinterpret_cast<cplx_t<T> *>(H));
    return hipGetLastError();
}

template <typename T>
hipError_t vec_symbol(const SpecCtx &c, int op, const double *x, const void *y, double a, int leray, double *out,
                      hipStream_t s) {
    const unsigned nb = (unsigned)((c.g.Nh() + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_vec_symbol<T>, dim3(nb), dim3(kThreads), 0, s, c.g, op,
                       reinterpret_cast<const double2 *>(x), reinterpret_cast<const cplx_t<T> *>(y), a, leray,
                       reinterpret_cast<double2 *>(out));
    return hipGetLastError();
}

hipError_t vec_dot_partials(const SpecCtx &c, int mode, const double *a, const double *b, double *partials,
                            int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_vec_dot<double2>, dim3(nblocks), dim3(kThreads), 0, s, c.g, mode,
                       reinterpret_cast<const double2 *>(a), reinterpret_cast<const double2 *>(b ? b : a), partials);
    return hipGetLastError();
}

template <typename T>
hipError_t krylov_dot_partials(const SpecCtx &c, const double *a, const void *b, double *partials, int nblocks,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_vec_dot<cplx_t<T>>, dim3(nblocks), dim3(kThreads), 0, s, c.g, 0,
                       reinterpret_cast<const double2 *>(a), reinterpret_cast<const cplx_t<T> *>(b), partials);
    return hipGetLastError();
}

template <typename T>
hipError_t krylov_axpy(const SpecCtx &c, const double *x, double a, const void *y, double *out, hipStream_t s) {
    const long n = 3 * c.g.Nh();
    hipLaunchKernelGGL(k_vec_axpy_krylov<T>, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n,
                       reinterpret_cast<const double2 *>(x), a, reinterpret_cast<const cplx_t<T> *>(y),
                       reinterpret_cast<double2 *>(out));
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_start(const SpecCtx &c, const double *g, double beta, int leray, void *s, void *r, void *p,
                     double *part_rz, int nblocks, hipStream_t st) {
    using C = cplx_t<T>;
    hipLaunchKernelGGL(k_pcg_start<T>, dim3(nblocks), dim3(kThreads), 0, st, c.g,
                       reinterpret_cast<const double2 *>(g), beta, leray, reinterpret_cast<C *>(s),
                       reinterpret_cast<C *>(r), reinterpret_cast<C *>(p), part_rz);
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_step(const SpecCtx &c, double a, const void *p, const void *y, double beta, int leray, void *s, void *r,
                    double *part_rr, double *part_rz, int nblocks, hipStream_t st) {
    using C = cplx_t<T>;
    hipLaunchKernelGGL(k_pcg_step<T>, dim3(nblocks), dim3(kThreads), 0, st, c.g, a, reinterpret_cast<const C *>(p),
                       reinterpret_cast<const C *>(y), beta, leray, reinterpret_cast<C *>(s), reinterpret_cast<C *>(r),
                       part_rr, part_rz);
    return hipGetLastError();
}

template <typename T>
hipError_t pcg_direction(const SpecCtx &c, const void *r, double b, double beta, int leray, void *p, hipStream_t st) {
    using C = cplx_t<T>;
    const unsigned nb = (unsigned)((c.g.Nh() + kThreads - 1) / kThreads);
    hipLaunchKernelGGL(k_pcg_direction<T>, dim3(nb), dim3(kThreads), 0, st, c.g, reinterpret_cast<const C *>(r), b,
                       beta, leray, reinterpret_cast<C *>(p));
    return hipGetLastError();
}

template <typename T>
hipError_t vec_assemble_dot(const SpecCtx &c, const double *x, const void *y, double a, int leray, int dot, double *out,
                            double *part, int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_vec_assemble_dot<T, double2>), dim3(nblocks), dim3(kThreads), 0, st, c.g,
                       reinterpret_cast<const double2 *>(x), reinterpret_cast<const cplx_t<T> *>(y), a, leray, dot,
                       reinterpret_cast<double2 *>(out), part);
    return hipGetLastError();
}

template <typename T>
hipError_t krylov_curvature(const SpecCtx &c, const void *p, const void *y, double beta, int leray, double *part,
                            int nblocks, hipStream_t st) {
    hipLaunchKernelGGL((k_vec_assemble_dot<T, cplx_t<T>>), dim3(nblocks), dim3(kThreads), 0, st, c.g,
                       reinterpret_cast<const cplx_t<T> *>(p), reinterpret_cast<const cplx_t<T> *>(y), beta, leray, 1,
                       nullptr, part);
    return hipGetLastError();
}

#define REGK_FFT_INST(T)                                                                                           \
    template hipError_t spec_resample<T>(const SpecCtx &, const SpecCtx &, int, hipStream_t);                     \
    template hipError_t spec_deriv<T>(const SpecCtx &, int, const T *, long, T *, long, int, int, hipStream_t);    \
    template hipError_t spec_forward<T, T>(const SpecCtx &, const T *, int, int, hipStream_t);                     \
    template hipError_t spec_inverse<T, T>(const SpecCtx &, T *, int, hipStream_t);                                \
    template hipError_t spec_symbol<T>(const SpecCtx &, int, double, int, int, hipStream_t);                       \
    template hipError_t spec_forward_to<T, T>(const SpecCtx &, const T *, int, void *, hipStream_t);              \
    template hipError_t spec_inverse_from<T, T>(const SpecCtx &, void *, T *, int, hipStream_t, const void *);    \
    template hipError_t vec_load<T>(const SpecCtx &, const double *, void *, hipStream_t);                         \
    template hipError_t vec_assemble_dot<T>(const SpecCtx &, const double *, const void *, double, int, int,        \
                                            double *, double *, int, hipStream_t);                                  \
    template hipError_t pcg_start<T>(const SpecCtx &, const double *, double, int, void *, void *, void *,        \
                                     double *, int, hipStream_t);                                                   \
    template hipError_t pcg_step<T>(const SpecCtx &, double, const void *, const void *, double, int, void *,      \
                                    void *, double *, double *, int, hipStream_t);                                  \
    template hipError_t pcg_direction<T>(const SpecCtx &, const void *, double, double, int, void *, hipStream_t); \
    template hipError_t krylov_curvature<T>(const SpecCtx &, const void *, const void *, double, int, double *,     \
                                            int, hipStream_t);                                                      \
    template hipError_t krylov_dot_partials<T>(const SpecCtx &, const double *, const void *, double *, int,       \
                                               hipStream_t);                                                        \
    template hipError_t krylov_axpy<T>(const SpecCtx &, const double *, double, const void *, double *,            \
                                       hipStream_t);                                                                \
    template hipError_t vec_symbol<T>(const SpecCtx &, int, const double *, const void *, double, int, double *,  \
                                      hipStream_t);

REGK_FFT_INST(float)
REGK_FFT_INST(double)
template hipError_t spec_forward<float, double>(const SpecCtx &, const float *, int, int, hipStream_t);

}  // namespace regk
