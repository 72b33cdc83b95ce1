// Host side of the learned warm start (reg_net_*, reg_warmstart): the
// network's layers, its workspace, forward and backward passes, the Adam
// step, and the warm start of a registration context.
//
// Network on an n^3 grid (n = 64 in use), activations BF16 channel-last:
//   e1a = relu(conv(x, 2->16)),  e1 = relu(conv(e1a, 16->16))        n^3
//   d2  = relu(conv_s2(e1, 16->32)), e2 = relu(conv(d2, 32->32))      (n/2)^3
//   d3  = relu(conv_s2(e2, 32->64)), b1, b2 = relu(conv(., 64->64))   (n/4)^3
//   u2  = relu(conv(up2(b2), 64->32)), m2 = relu(conv([u2, e2], 64->32))
//   u1  = relu(conv(up2(m2), 32->16)), m1 = relu(conv([u1, e1], 32->16))
//   v   = conv(m1, 16->3)
// The concatenations are free: u2 and e2 are written into the two channel
// halves of one buffer (cat2), u1 and e1 into cat1.
//
// Warm start: the context's images are resampled spectrally to n^3, the
// network proposes v there, v is resampled back to the context's grid,
// projected when isochoric, and accepted only if det(grad y1) > 0 everywhere;
// otherwise the caller gets v = 0 (cold start).
#include <algorithm>
#include <cmath>

#include "ctx.hpp"
#include "net.hpp"

using namespace regc;

namespace {

struct LayerDef {
    int cin, cout, stride;
};
constexpr int kLayers = 12;
constexpr LayerDef kDef[kLayers] = {{2, 16, 1},  {16, 16, 1}, {16, 32, 2}, {32, 32, 1}, {32, 64, 2}, {64, 64, 1},
                                    {64, 64, 1}, {64, 32, 1}, {64, 32, 1}, {32, 16, 1}, {32, 16, 1}, {16, 3, 1}};

int pad16(int c) { return (c + 15) / 16 * 16; }

long param_count() {
    long n = 0;
    for (const auto &L : kDef) n += (long)L.cout * L.cin * 27 + L.cout;
    return n;
}

bool net_grid_ok(int n) { return n >= 16 && n <= 256 && n % 16 == 0 && fft_friendly(n); }

}  // namespace

struct reg_net {
    int n = 0;
    long P1 = 0, P2 = 0, P3 = 0;
    hipStream_t stream = nullptr;
    long count = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    long woff[kLayers], boff[kLayers];
    uint16_t *wf[kLayers], *wb[kLayers];  // BF16 copies: [27][cout_pad][cin_pad], [27][cin_pad][cout_pad]
    // activations
    uint16_t *x0, *e1a, *cat1, *d2, *cat2, *d3, *b1, *b2, *upb2, *m2, *upm2, *m1;
    float *v;
    // gradients
    uint16_t *dz11, *dz10, *dcat1, *dz9, *dupm2, *dz8, *dcat2, *dz7, *dupb2, *dz6, *dz5, *dz4, *dz3, *dz2, *dz1, *dz0;
    float *partials = nullptr, *bias_partials = nullptr;
    double *mse_part = nullptr, *loss = nullptr;
    double *hloss = nullptr;  // pinned
    int step = 0;
    bool weights_packed = false;
    bool have_forward = false;  // activations of a reg_net_forward are in place
    // warm start: a single-precision context on the network grid (spectral
    // resampling) and the network's input / output fields there
    reg_ctx *rctx = nullptr;
    void *rws = nullptr;  // its workspace
    float *rT = nullptr, *rR = nullptr;
    std::string err;
};

namespace {

reg_status nfail(reg_net *net, reg_status st, const std::string &msg) {
    if (net) net->err = msg;
    return st;
}

#define NHIP(net, expr)                                                                 \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) return nfail((net), REG_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

reg_params resample_params(int n) {
    reg_params p;
    reg_default_params(&p);
    p.n[0] = p.n[1] = p.n[2] = n;
    p.nt = 1;
    p.prec = 0;
    return p;
}

size_t net_layout(int n, char *base, reg_net *net) {
    Layout L(base);
    reg_net tmp;
    reg_net *t = net ? net : &tmp;
    const long P1 = (long)n * n * n, P2 = P1 / 8, P3 = P1 / 64;
    const long cnt = param_count();
    t->params = (float *)L.take(sizeof(float) * cnt);
    t->grads = (float *)L.take(sizeof(float) * cnt);
    t->adam_m = (float *)L.take(sizeof(float) * cnt);
    t->adam_v = (float *)L.take(sizeof(float) * cnt);
    for (int l = 0; l < kLayers; l++) {
        const size_t e = 27 * (size_t)pad16(kDef[l].cout) * pad16(kDef[l].cin);
        t->wf[l] = (uint16_t *)L.take(2 * e);
        t->wb[l] = (uint16_t *)L.take(2 * e);
    }
    auto act = [&](long P, int C) { return (uint16_t *)L.take(2 * (size_t)P * C); };
    t->x0 = act(P1, 16);
    t->e1a = act(P1, 16);
    t->cat1 = act(P1, 32);
    t->d2 = act(P2, 32);
    t->cat2 = act(P2, 64);
    t->d3 = act(P3, 64);
    t->b1 = act(P3, 64);
    t->b2 = act(P3, 64);
    t->upb2 = act(P2, 64);
    t->m2 = act(P2, 32);
    t->upm2 = act(P1, 32);
    t->m1 = act(P1, 16);
    t->v = (float *)L.take(sizeof(float) * 3 * P1);
    t->dz11 = act(P1, 16);
    t->dz10 = act(P1, 16);
    t->dcat1 = act(P1, 32);
    t->dz9 = act(P1, 16);
    t->dupm2 = act(P1, 32);
    t->dz8 = act(P2, 32);
    t->dcat2 = act(P2, 64);
    t->dz7 = act(P2, 32);
    t->dupb2 = act(P2, 64);
    t->dz6 = act(P3, 64);
    t->dz5 = act(P3, 64);
    t->dz4 = act(P3, 64);
    t->dz3 = act(P2, 32);
    t->dz2 = act(P2, 32);
    t->dz1 = act(P1, 16);
    t->dz0 = act(P1, 16);
    size_t part = 0, bpart = 0;
    for (int l = 0; l < kLayers; l++) {
        const int no = (l >= 2 && l <= 3) || l == 7 || l == 8 ? n / 2 : (l >= 4 && l <= 6) ? n / 4 : n;
        part = std::max(part, (size_t)regn::wgrad_chunks(no) * 27 * pad16(kDef[l].cout) * pad16(kDef[l].cin));
        bpart = std::max(bpart, (size_t)regn::wgrad_chunks(no) * pad16(kDef[l].cout));
    }
    t->partials = (float *)L.take(sizeof(float) * part);
    t->bias_partials = (float *)L.take(sizeof(float) * bpart);
    t->mse_part = (double *)L.take(sizeof(double) * regn::mse_blocks(P1));
    t->loss = (double *)L.take(sizeof(double));
    t->rT = (float *)L.take(sizeof(float) * P1);
    t->rR = (float *)L.take(sizeof(float) * P1);
    size_t rbytes = 0;
    reg_params rp = resample_params(n);
    reg_workspace_size(&rp, &rbytes);
    t->rws = L.take(rbytes);
    return L.off;
}

// grid of layer l's output
int out_grid(const reg_net *net, int l) {
    if (l >= 4 && l <= 6) return net->n / 4;
    if ((l >= 2 && l <= 3) || l == 7 || l == 8) return net->n / 2;
    return net->n;
}

reg_status pack_weights(reg_net *net) {
    for (int l = 0; l < kLayers; l++)
        NHIP(net, regn::launch_pack_weights(net->params + net->woff[l], kDef[l].cout, kDef[l].cin, pad16(kDef[l].cout),
                                            pad16(kDef[l].cin), net->wf[l], net->wb[l], net->stream));
    net->weights_packed = true;
    return REG_OK;
}

// forward convolution of layer l from `in` (channel stride in_cs) into `out`
reg_status conv_fwd(reg_net *net, int l, const uint16_t *in, int in_cs, uint16_t *out, int out_cs, bool relu,
                    float *out_f32 = nullptr) {
    regn::ConvArgs a{};
    a.in = in;
    a.in_cs = in_cs;
    a.cin = pad16(kDef[l].cin);
    a.n_out = out_grid(net, l);
    a.n_in = kDef[l].stride == 2 ? 2 * a.n_out : a.n_out;
    a.w = net->wf[l];
    a.cout = pad16(kDef[l].cout);
    a.bias = net->params + net->boff[l];
    a.relu = relu;
    a.out = out;
    a.out_cs = out_cs;
    a.out_f32 = out_f32;
    a.cout_real = kDef[l].cout;  // padded channels get no bias
    NHIP(net, regn::launch_conv(kDef[l].stride == 2 ? regn::CONV_FWD2 : regn::CONV_FWD1, a, net->stream));
    return REG_OK;
}

reg_status forward(reg_net *net, const float *rhoT, const float *rhoR) {
    if (!net->weights_packed) STCHK(pack_weights(net));
    const long P1 = net->P1;
    NHIP(net, regn::launch_pack_input(rhoT, rhoR, P1, net->x0, net->stream));
    STCHK(conv_fwd(net, 0, net->x0, 16, net->e1a, 16, true));
    STCHK(conv_fwd(net, 1, net->e1a, 16, net->cat1 + 16, 32, true));
    STCHK(conv_fwd(net, 2, net->cat1 + 16, 32, net->d2, 32, true));
    STCHK(conv_fwd(net, 3, net->d2, 32, net->cat2 + 32, 64, true));
    STCHK(conv_fwd(net, 4, net->cat2 + 32, 64, net->d3, 64, true));
    STCHK(conv_fwd(net, 5, net->d3, 64, net->b1, 64, true));
    STCHK(conv_fwd(net, 6, net->b1, 64, net->b2, 64, true));
    NHIP(net, regn::launch_up2(net->b2, net->n / 4, 64, net->upb2, net->stream));
    STCHK(conv_fwd(net, 7, net->upb2, 64, net->cat2, 64, true));
    STCHK(conv_fwd(net, 8, net->cat2, 64, net->m2, 32, true));
    NHIP(net, regn::launch_up2(net->m2, net->n / 2, 32, net->upm2, net->stream));
    STCHK(conv_fwd(net, 9, net->upm2, 32, net->cat1, 32, true));
    STCHK(conv_fwd(net, 10, net->cat1, 32, net->m1, 16, true));
    STCHK(conv_fwd(net, 11, net->m1, 16, nullptr, 0, false, net->v));  // head: FP32 [3][P]
    return REG_OK;
}

// backward-data of layer l: dz (its output-side gradient, pad16(cout)
// channels) to the gradient of its input (pad16(cin) channels)
reg_status conv_bwd(reg_net *net, int l, const uint16_t *dz, uint16_t *out, int out_cs, const uint16_t *mask,
                    int mask_cs, const uint16_t *add = nullptr, int add_cs = 0) {
    regn::ConvArgs a{};
    a.in = dz;
    a.in_cs = pad16(kDef[l].cout);
    a.cin = pad16(kDef[l].cout);
    const int no = out_grid(net, l);
    a.n_in = no;
    a.n_out = kDef[l].stride == 2 ? 2 * no : no;
    a.w = net->wb[l];
    a.cout = pad16(kDef[l].cin);
    a.add = add;
    a.add_cs = add_cs;
    a.mask = mask;
    a.mask_cs = mask_cs;
    a.out = out;
    a.out_cs = out_cs;
    a.cout_real = a.cout;
    NHIP(net, regn::launch_conv(kDef[l].stride == 2 ? regn::CONV_BWD2 : regn::CONV_BWD1, a, net->stream));
    return REG_OK;
}

// weight and bias gradients of layer l (accumulated with `scale`)
reg_status wgrad(reg_net *net, int l, const uint16_t *x, int x_cs, const uint16_t *dz, float scale) {
    regn::WgradArgs a{};
    a.dz = dz;
    a.dz_cs = pad16(kDef[l].cout);
    a.cout = pad16(kDef[l].cout);
    a.x = x;
    a.x_cs = x_cs;
    a.cin = pad16(kDef[l].cin);
    a.n_out = out_grid(net, l);
    a.n_in = kDef[l].stride == 2 ? 2 * a.n_out : a.n_out;
    a.partials = net->partials;
    a.bias_partials = net->bias_partials;
    const int mode = kDef[l].stride == 2 ? regn::CONV_FWD2 : regn::CONV_FWD1;
    NHIP(net, regn::launch_wgrad(mode, a, net->stream));
    NHIP(net, regn::launch_wgrad_reduce(net->partials, net->bias_partials, regn::wgrad_chunks(a.n_out), a.cout, a.cin,
                                        kDef[l].cout, kDef[l].cin, scale, net->grads + net->woff[l],
                                        net->grads + net->boff[l], net->stream));
    return REG_OK;
}

// the backward pass from the head's pre-activation gradient in dz11 (the
// gradient of one sample's loss); the batch weight `scale` enters the weight
// and bias reductions
reg_status backward_from_head(reg_net *net, float scale) {
    const long P1 = net->P1, P2 = net->P2;
    STCHK(wgrad(net, 11, net->m1, 16, net->dz11, scale));
    STCHK(conv_bwd(net, 11, net->dz11, net->dz10, 16, net->m1, 16));
    STCHK(wgrad(net, 10, net->cat1, 32, net->dz10, scale));
    STCHK(conv_bwd(net, 10, net->dz10, net->dcat1, 32, nullptr, 0));
    NHIP(net, regn::launch_mask(net->dcat1, 32, P1, 16, net->cat1, 32, net->dz9, net->stream));
    STCHK(wgrad(net, 9, net->upm2, 32, net->dz9, scale));
    STCHK(conv_bwd(net, 9, net->dz9, net->dupm2, 32, nullptr, 0));
    NHIP(net, regn::launch_up2_bwd(net->dupm2, net->n / 2, 32, net->m2, 32, net->dz8, net->stream));
    STCHK(wgrad(net, 8, net->cat2, 64, net->dz8, scale));
    STCHK(conv_bwd(net, 8, net->dz8, net->dcat2, 64, nullptr, 0));
    NHIP(net, regn::launch_mask(net->dcat2, 64, P2, 32, net->cat2, 64, net->dz7, net->stream));
    STCHK(wgrad(net, 7, net->upb2, 64, net->dz7, scale));
    STCHK(conv_bwd(net, 7, net->dz7, net->dupb2, 64, nullptr, 0));
    NHIP(net, regn::launch_up2_bwd(net->dupb2, net->n / 4, 64, net->b2, 64, net->dz6, net->stream));
    STCHK(wgrad(net, 6, net->b1, 64, net->dz6, scale));
    STCHK(conv_bwd(net, 6, net->dz6, net->dz5, 64, net->b1, 64));
    STCHK(wgrad(net, 5, net->d3, 64, net->dz5, scale));
    STCHK(conv_bwd(net, 5, net->dz5, net->dz4, 64, net->d3, 64));
    STCHK(wgrad(net, 4, net->cat2 + 32, 64, net->dz4, scale));
    // e2 collects the stride-2 path and the skip half of dcat2
    STCHK(conv_bwd(net, 4, net->dz4, net->dz3, 32, net->cat2 + 32, 64, net->dcat2 + 32, 64));
    STCHK(wgrad(net, 3, net->d2, 32, net->dz3, scale));
    STCHK(conv_bwd(net, 3, net->dz3, net->dz2, 32, net->d2, 32));
    STCHK(wgrad(net, 2, net->cat1 + 16, 32, net->dz2, scale));
    // e1 collects the stride-2 path and the skip half of dcat1
    STCHK(conv_bwd(net, 2, net->dz2, net->dz1, 16, net->cat1 + 16, 32, net->dcat1 + 16, 32));
    STCHK(wgrad(net, 1, net->e1a, 16, net->dz1, scale));
    STCHK(conv_bwd(net, 1, net->dz1, net->dz0, 16, net->e1a, 16));
    STCHK(wgrad(net, 0, net->x0, 16, net->dz0, scale));
    return REG_OK;
}

// the MSE loss of the last forward pass against `target` and its backward
// pass: loss and parameter gradients of one sample, accumulated into loss and
// grads with weight `scale`
reg_status backward(reg_net *net, const float *target, float scale) {
    NHIP(net, regn::launch_mse(net->v, target, net->P1, net->mse_part, net->loss, scale / (3.0 * net->P1), net->dz11,
                               net->stream));
    return backward_from_head(net, scale);
}

#define NET_OK(net)                                   \
    do {                                              \
        if (!(net)) return REG_EINVAL;                \
        (net)->err.clear();                           \
    } while (0)

#define NET_DEV(net, ptr)                                                                           \
    do {                                                                                            \
        if (!is_device_ptr(ptr)) return nfail((net), REG_EINVAL, #ptr " is not a device pointer");  \
    } while (0)

}  // namespace

extern "C" {

reg_status reg_net_param_count(int64_t *count) {
    if (!count) return REG_EINVAL;
    *count = param_count();
    return REG_OK;
}

reg_status reg_net_workspace_size(int32_t n, size_t *bytes) {
    if (!bytes || !net_grid_ok(n)) return REG_EINVAL;
    *bytes = net_layout(n, nullptr, nullptr);
    return REG_OK;
}

reg_status reg_net_create(int32_t n, void *workspace, size_t bytes, void *hip_stream, reg_net **out) {
    if (!out) return REG_EINVAL;
    *out = nullptr;
    if (!net_grid_ok(n)) return REG_EINVAL;
    if (!workspace || ((uintptr_t)workspace % kAlign) != 0 || !is_device_ptr(workspace)) return REG_EINVAL;
    if (bytes < net_layout(n, nullptr, nullptr)) return REG_ENOMEM;
    reg_net *net = new (std::nothrow) reg_net();
    if (!net) return REG_ENOMEM;
    net->n = n;
    net->P1 = (long)n * n * n;
    net->P2 = net->P1 / 8;
    net->P3 = net->P1 / 64;
    net->stream = (hipStream_t)hip_stream;
    net->count = param_count();
    long off = 0;
    for (int l = 0; l < kLayers; l++) {
        net->woff[l] = off;
        off += (long)kDef[l].cout * kDef[l].cin * 27;
        net->boff[l] = off;
        off += kDef[l].cout;
    }
    net_layout(n, (char *)workspace, net);
    reg_params rp = resample_params(n);
    size_t rbytes = 0;
    reg_workspace_size(&rp, &rbytes);
    if (hipHostMalloc((void **)&net->hloss, sizeof(double), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete net;
        return REG_EHIP;
    }
    reg_status st = reg_create(&rp, net->rws, rbytes, hip_stream, &net->rctx);
    if (st != REG_OK) {
        (void)hipHostFree(net->hloss);
        delete net;
        return st;
    }
    // zero parameters, gradients and moments until set
    if (regn::launch_fill_f32(net->count, 0.f, net->params, net->stream) != hipSuccess ||
        regn::launch_fill_f32(net->count, 0.f, net->grads, net->stream) != hipSuccess ||
        regn::launch_fill_f32(net->count, 0.f, net->adam_m, net->stream) != hipSuccess ||
        regn::launch_fill_f32(net->count, 0.f, net->adam_v, net->stream) != hipSuccess) {
        reg_destroy(net->rctx);
        (void)hipHostFree(net->hloss);
        delete net;
        return REG_EHIP;
    }
    *out = net;
    return REG_OK;
}

reg_status reg_net_destroy(reg_net *net) {
    if (!net) return REG_EINVAL;
    (void)hipStreamSynchronize(net->stream);
    if (net->rctx) reg_destroy(net->rctx);
    if (net->hloss) (void)hipHostFree(net->hloss);
    delete net;
    return REG_OK;
}

const char *reg_net_last_error(const reg_net *net) { return net ? net->err.c_str() : "null network"; }

reg_status reg_net_set_params(reg_net *net, const float *params) {
    NET_OK(net);
    NET_DEV(net, params);
    net->have_forward = false;
    NHIP(net, hipMemcpyAsync(net->params, params, sizeof(float) * net->count, hipMemcpyDeviceToDevice, net->stream));
    NHIP(net, regn::launch_fill_f32(net->count, 0.f, net->adam_m, net->stream));
    NHIP(net, regn::launch_fill_f32(net->count, 0.f, net->adam_v, net->stream));
    net->step = 0;
    return pack_weights(net);
}

reg_status reg_net_get_params(reg_net *net, float *params) {
    NET_OK(net);
    NET_DEV(net, params);
    NHIP(net, hipMemcpyAsync(params, net->params, sizeof(float) * net->count, hipMemcpyDeviceToDevice, net->stream));
    return REG_OK;
}

reg_status reg_net_forward(reg_net *net, const float *rhoT, const float *rhoR, float *v) {
    NET_OK(net);
    NET_DEV(net, rhoT);
    NET_DEV(net, rhoR);
    NET_DEV(net, v);
    net->have_forward = false;
    STCHK(forward(net, rhoT, rhoR));
    NHIP(net, hipMemcpyAsync(v, net->v, sizeof(float) * 3 * net->P1, hipMemcpyDeviceToDevice, net->stream));
    net->have_forward = true;
    return REG_OK;
}

reg_status reg_net_activation(reg_net *net, int32_t layer, float *out) {
    NET_OK(net);
    NET_DEV(net, out);
    if (layer < 0 || layer >= kLayers) return nfail(net, REG_EINVAL, "layer must be 0..11");
    const uint16_t *src[kLayers] = {net->e1a, net->cat1 + 16, net->d2, net->cat2 + 32, net->d3, net->b1,
                                    net->b2, net->cat2, net->m2, net->cat1, net->m1, nullptr};
    const int cs[kLayers] = {16, 32, 32, 64, 64, 64, 64, 64, 32, 32, 16, 0};
    const int no = out_grid(net, layer);
    const long P = (long)no * no * no;
    if (layer == kLayers - 1) {
        NHIP(net, hipMemcpyAsync(out, net->v, sizeof(float) * 3 * P, hipMemcpyDeviceToDevice, net->stream));
        return REG_OK;
    }
    NHIP(net, regn::launch_unpack(src[layer], cs[layer], kDef[layer].cout, P, out, net->stream));
    return REG_OK;
}

reg_status reg_net_loss_grad(reg_net *net, const float *rhoT, const float *rhoR, const float *target, float *grad,
                             double *loss) {
    NET_OK(net);
    NET_DEV(net, rhoT);
    NET_DEV(net, rhoR);
    NET_DEV(net, target);
    NET_DEV(net, grad);
    if (!loss) return nfail(net, REG_EINVAL, "loss is NULL");
    net->have_forward = false;
    NHIP(net, regn::launch_fill_f32(net->count, 0.f, net->grads, net->stream));
    NHIP(net, regk::launch_fill<double>(1, 0.0, net->loss, net->stream));
    STCHK(forward(net, rhoT, rhoR));
    STCHK(backward(net, target, 1.f));
    NHIP(net, hipMemcpyAsync(grad, net->grads, sizeof(float) * net->count, hipMemcpyDeviceToDevice, net->stream));
    NHIP(net, hipMemcpyAsync(net->hloss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->stream));
    NHIP(net, hipStreamSynchronize(net->stream));
    *loss = *net->hloss;
    return REG_OK;
}

reg_status reg_net_backward(reg_net *net, const float *dv, float *grad) {
    NET_OK(net);
    NET_DEV(net, dv);
    NET_DEV(net, grad);
    if (!net->have_forward) return nfail(net, REG_EINVAL, "reg_net_backward needs a reg_net_forward before it");
    NHIP(net, regn::launch_fill_f32(net->count, 0.f, net->grads, net->stream));
    NHIP(net, regn::launch_pack_head_grad(dv, net->P1, 1.f, net->dz11, net->stream));
    STCHK(backward_from_head(net, 1.f));
    NHIP(net, hipMemcpyAsync(grad, net->grads, sizeof(float) * net->count, hipMemcpyDeviceToDevice, net->stream));
    NHIP(net, hipStreamSynchronize(net->stream));
    return REG_OK;
}

reg_status reg_net_step(reg_net *net, const float *grad, double lr) {
    NET_OK(net);
    NET_DEV(net, grad);
    if (!(lr > 0) || !std::isfinite(lr)) return nfail(net, REG_EINVAL, "lr must be positive");
    NHIP(net, hipMemcpyAsync(net->grads, grad, sizeof(float) * net->count, hipMemcpyDeviceToDevice, net->stream));
    net->step++;
    NHIP(net, regn::launch_adam(net->count, net->params, net->grads, net->adam_m, net->adam_v, (float)lr, 0.9f, 0.999f,
                                1e-8f, net->step, net->stream));
    STCHK(pack_weights(net));
    net->have_forward = false;
    NHIP(net, hipStreamSynchronize(net->stream));
    return REG_OK;
}

reg_status reg_net_train_step(reg_net *net, int32_t batch, const float *const *rhoT, const float *const *rhoR,
                              const float *const *target, double lr, double *loss) {
    NET_OK(net);
    net->have_forward = false;
    if (batch < 1 || !rhoT || !rhoR || !target || !loss) return nfail(net, REG_EINVAL, "bad batch arguments");
    if (!(lr > 0) || !std::isfinite(lr)) return nfail(net, REG_EINVAL, "lr must be positive");
    for (int b = 0; b < batch; b++) {
        NET_DEV(net, rhoT[b]);
        NET_DEV(net, rhoR[b]);
        NET_DEV(net, target[b]);
    }
    NHIP(net, regn::launch_fill_f32(net->count, 0.f, net->grads, net->stream));
    NHIP(net, regk::launch_fill<double>(1, 0.0, net->loss, net->stream));
    const float scale = 1.f / batch;
    for (int b = 0; b < batch; b++) {
        STCHK(forward(net, rhoT[b], rhoR[b]));
        STCHK(backward(net, target[b], scale));
    }
    net->step++;
    NHIP(net, regn::launch_adam(net->count, net->params, net->grads, net->adam_m, net->adam_v, (float)lr, 0.9f, 0.999f,
                                1e-8f, net->step, net->stream));
    STCHK(pack_weights(net));
    NHIP(net, hipMemcpyAsync(net->hloss, net->loss, sizeof(double), hipMemcpyDeviceToHost, net->stream));
    NHIP(net, hipStreamSynchronize(net->stream));
    *loss = *net->hloss;
    if (!std::isfinite(*loss)) return nfail(net, REG_ENONFINITE, "non-finite training loss");
    return REG_OK;
}

reg_status reg_warmstart(reg_ctx *ctx, reg_net *net, void *v_out, int32_t *used_fallback, double *detmin) {
    CTX_OK(ctx);
    if (!net) return fail(ctx, REG_EINVAL, "net is NULL");
    net->have_forward = false;
    NEED_DEV(ctx, v_out);
    if (!used_fallback) return fail(ctx, REG_EINVAL, "used_fallback is NULL");
    if (ctx->P.prec != 0) return fail(ctx, REG_EINVAL, "the warm start needs a single-precision context");
    if (!ctx->have_images) return fail(ctx, REG_EINVAL, "reg_set_images has not been called");
    const long N3 = 3 * ctx->N;
    // images to the network grid (on the context's stream), the network (on
    // its own), the velocity back to the context's grid; the streams are
    // joined by synchronisation between the stages
    STCHK(reg_resample(ctx, net->rctx, 1, ctx->rhoT, net->rT));
    STCHK(reg_resample(ctx, net->rctx, 1, ctx->rhoR, net->rR));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    reg_status st = forward(net, net->rT, net->rR);
    if (st != REG_OK) return fail(ctx, st, "network forward: " + net->err);
    HIPCHK(ctx, hipStreamSynchronize(net->stream));
    st = reg_resample(net->rctx, ctx, 3, net->v, ctx->vf);
    if (st != REG_OK) return fail(ctx, st, std::string("resampling the proposed velocity: ") + reg_last_error(net->rctx));
    HIPCHK(ctx, hipStreamSynchronize(net->stream));
    HIPCHK(ctx, KL(ctx, REG_K_VECTOR, (regk::launch_convert<float, double>(N3, CV<float>(ctx->vf), V<double>(v_out), ctx->stream))));
    if (ctx->P.isochoric) {
        HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_forward<double, double>(ctx->spec, CV<double>(v_out), 3, 0, ctx->stream))));
        HIPCHK(ctx, KL(ctx, REG_K_SYMBOL, regk::spec_symbol<double>(ctx->spec, regk::SYM_LERAY, 0.0, 3, 1, ctx->stream)));
        HIPCHK(ctx, KL(ctx, REG_K_FFT3D, (regk::spec_inverse<double, double>(ctx->spec, V<double>(v_out), 3, ctx->stream))));
    }
    // the solver decides: accept the proposal only if its map is a
    // diffeomorphism on the grid (det grad y1 > 0 everywhere)
    double dmin = 0, dmax = 0;
    STCHK(reg_deformation(ctx, v_out, nullptr, &dmin, &dmax));
    if (detmin) *detmin = dmin;
    const bool ok = std::isfinite(dmin) && std::isfinite(dmax) && dmin > 0;
    *used_fallback = ok ? 0 : 1;
    if (!ok) {
        HIPCHK(ctx, KL(ctx, REG_K_VECTOR, regk::launch_fill<double>(N3, 0.0, V<double>(v_out), ctx->stream)));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    return REG_OK;
}

}  // extern "C"
