// Context-free periodic tricubic interpolation that allocates nothing: the
// variant of reg_interp for callers that cannot allocate device memory.
// reg_interp keeps the floor-bound partials of the departure points (from
// which the LDS tile geometry of the gather is chosen) in its context's
// workspace; here they live in a file-scope device array of fixed size, one
// copy per GPU, whose device address is looked up once per device.
#include <mutex>

#include "ctx.hpp"

namespace {

constexpr int kBoundBlocks = regk::RED_BLOCKS / 6;  // blocks of the floor-bound reduction
constexpr int kBoundsAt = 6 * kBoundBlocks;         // the six reduced bounds follow the partials
constexpr int kScratchDoubles = kBoundsAt + 6;      // 1026 doubles, about 8 KiB per GPU
constexpr int kMaxDevices = 64;

// Partial and final floor bounds of D. Host code never uses this name as an
// address: it passes the per-device pointer from hipGetSymbolAddress.
static __device__ __align__(256) double scratch[kScratchDoubles];

std::mutex g_mutex;
double *g_scratch[kMaxDevices];  // device address of `scratch` on each device, once looked up

// The scratch address on the current device `dev` (looked up on the first
// call there).
reg_status scratch_on(int dev, double **out) {
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            std::fprintf(stderr, "reg_interp_noalloc: hipGetSymbolAddress failed on device %d: %s\n", dev,
                         hipGetErrorString(e));
            return REG_EHIP;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return REG_OK;
}

reg_status reject(const char *why) {
    std::fprintf(stderr, "reg_interp_noalloc: %s\n", why);
    return REG_EINVAL;
}

bool on_device(const void *p, int dev) {
    if (!p) return false;
    hipPointerAttribute_t a;
    if (hipPointerGetAttributes(&a, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return (a.type == hipMemoryTypeDevice || a.type == hipMemoryTypeManaged) && a.device == dev;
}

template <typename T>
reg_status interp(const regk::Grid &g, const void *f, const void *D, void *out, double *s, hipStream_t st) {
    const T *Dt = static_cast<const T *>(D);
    if (regk::launch_floor_bounds<T>(g, Dt, s, kBoundBlocks, st) != hipSuccess ||
        regk::launch_finalize_bounds(s, kBoundBlocks, s + kBoundsAt, st) != hipSuccess)
        return REG_EHIP;
    double b[6];
    if (hipMemcpyAsync(b, s + kBoundsAt, sizeof(b), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
        (void)hipGetLastError();
        return REG_EHIP;
    }
    const double fmin[3] = {b[0], b[2], b[4]}, fmax[3] = {b[1], b[3], b[5]};
    regk::TileGeom tg{};
    const bool tiled = regk::tile_geom(fmin, fmax, sizeof(T), &tg);
    if (regk::launch_interp<T>(g, static_cast<const T *>(f), Dt, static_cast<T *>(out), st, tiled ? &tg : nullptr) !=
        hipSuccess) {
        (void)hipGetLastError();
        return REG_EHIP;
    }
    return REG_OK;
}

}  // namespace

extern "C" reg_status reg_interp_noalloc(int32_t prec, const int32_t n[3], const void *f, const void *D, void *out,
                                         void *hip_stream) {
    if (prec != 0 && prec != 1) return reject("prec must be 0 (float) or 1 (double)");
    if (!n) return reject("n is NULL");
    for (int j = 0; j < 3; j++)
        if (!regc::fft_friendly(n[j])) return reject("each n[j] must be even, 2^a 3^b 5^c and in [8, 1024]");
    if (f == out) return reject("out must not alias f");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return REG_EHIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return reject("device index beyond the supported 64");
    if (!on_device(f, dev) || !on_device(D, dev) || !on_device(out, dev))
        return reject("f, D and out must be device pointers on the current device");
    double *s = nullptr;
    const reg_status st = scratch_on(dev, &s);
    if (st != REG_OK) return st;
    const regk::Grid g{n[0], n[1], n[2]};
    hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    return prec ? interp<double>(g, f, D, out, s, stream) : interp<float>(g, f, D, out, s, stream);
}
