// xrt_learn.cpp -- the U-Net preconditioner (parameters, workspace, forward,
// back-propagation, Adam) and the CG / flexible-PCG solvers of
// include/xrt_learn.h.  All arithmetic runs in the kernels of xrt_learn.hip
// and xrt_kernels.hip; this file only sequences launches on the caller's
// stream.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <random>
#include <vector>

#include "xrt.h"
#include "xrt_internal.h"
#include "xrt_learn.h"
#include "xrt_learn_internal.h"

using xrl::CView;
using xrl::View;

namespace {

constexpr uint64_t kNetMagic = 0x58525455'4e455431ull;  // "XRTUNET1"

struct Layer {
    int64_t off;    // offset in the fp32 parameter vector
    int64_t woff;   // offset in the bf16 weight arrays (elements, multiple of 64)
    int taps, cout, cin;
    int64_t size() const { return (int64_t)taps * cout * cin; }
};

// one bf16 NHWC buffer
struct Buf {
    uint16_t* p = nullptr;
    int c = 0;      // pitch (channels)
    View v(int off = 0) const { return View{p + off, c}; }
    CView cv(int off = 0) const { return CView{p + off, c}; }
};

}  // namespace

struct xrt_unet {
    uint64_t magic;
    int L, base, H, W, maxB;
    int ch[8];      // channels per level: min(base * 2^l, cap)
    std::vector<Layer> layers;
    int64_t nparam, nw;
    float *param, *grad, *m, *v;
    uint16_t *wf, *wb;
    int64_t step;
    float gain;     // fixed output gain: N(r) = gain * rms(r) * U(r / rms(r))
    bool relu;      // activation after every 3x3 convolution (false: a linear network)
    bool fuse = true;   // xrt_unet_apply reads pooled / upsampled inputs inside the convolutions
    // activations, per level (see forward())
    Buf in[8], eh[8], cat[8], ebot, uc[8], dh[8], dd[8];
    // gradients
    Buf gdd[8], gdh[8], gcat[8], guc[8], gebot, geh[8], gin[8];
    float *scale, *tn, *y, *gy, *lpart, *loss_tmp, *part;
    double* ipart;   // per-image reduction partials
    float* cws;      // split-K partial sums of the 3x3 convolutions
    int64_t cws_n;
    int64_t part_n;
    std::vector<void*> allocs;
};

namespace {

thread_local char g_err[256] = "";

xrt_status hip_fail(const char* what, hipError_t e)
{
    snprintf(g_err, sizeof(g_err), "%s: %s", what, hipGetErrorString(e));
    xrt::set_last_error(g_err);
    return XRT_EHIP;
}

#define XL_CHECK(call, what)                                   \
    do {                                                       \
        hipError_t e_ = (call);                                \
        if (e_ != hipSuccess) return hip_fail(what, e_);       \
    } while (0)

// The temporary buffers of one entry point, released on every return path:
// device buffers with hipFreeAsync on the entry point's stream, the pinned
// host buffer once that stream has drained (on an error path a copy into it
// may still be queued).
class Scratch {
public:
    explicit Scratch(hipStream_t s) : s_(s) {}
    Scratch(const Scratch&) = delete;
    Scratch& operator=(const Scratch&) = delete;
    template <typename T>
    hipError_t device(T** out, size_t bytes)
    {
        *out = nullptr;
        if (n_ == kMax) return hipErrorInvalidValue;
        void* p = nullptr;
        const hipError_t e = hipMallocAsync(&p, bytes, s_);
        if (e == hipSuccess) {
            dev_[n_++] = p;
            *out = (T*)p;
        }
        return e;
    }
    template <typename T>
    hipError_t host(T** out, size_t bytes)
    {
        *out = nullptr;
        if (host_) return hipErrorInvalidValue;
        void* p = nullptr;
        const hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocDefault);
        if (e == hipSuccess) {
            host_ = p;
            *out = (T*)p;
        }
        return e;
    }
    ~Scratch()
    {
        for (int i = n_ - 1; i >= 0; --i) (void)hipFreeAsync(dev_[i], s_);
        if (host_) {
            (void)hipStreamSynchronize(s_);
            (void)hipHostFree(host_);
        }
    }

private:
    static constexpr int kMax = 4;
    hipStream_t s_;
    void* dev_[kMax] = {};
    int n_ = 0;
    void* host_ = nullptr;
};

bool net_ok(const xrt_unet* n) { return n && n->magic == kNetMagic; }

int enc_a(const xrt_unet* n, int l) { (void)n; return 2 * l; }
int enc_b(const xrt_unet* n, int l) { (void)n; return 2 * l + 1; }
int dec_up(const xrt_unet* n, int l) { return 2 * n->L + 3 * (n->L - 2 - l); }
int dec_a(const xrt_unet* n, int l) { return dec_up(n, l) + 1; }
int dec_b(const xrt_unet* n, int l) { return dec_up(n, l) + 2; }
int out_layer(const xrt_unet* n) { return 2 * n->L + 3 * (n->L - 1); }

const uint16_t* WF(const xrt_unet* n, int k) { return n->wf + n->layers[k].woff; }
const uint16_t* WB(const xrt_unet* n, int k) { return n->wb + n->layers[k].woff; }

// encoder output of level l (a slice of the concatenation buffer below the bottleneck)
CView enc_out(const xrt_unet* n, int l) { return l == n->L - 1 ? n->ebot.cv() : n->cat[l].cv(); }
View enc_out_w(xrt_unet* n, int l) { return l == n->L - 1 ? n->ebot.v() : n->cat[l].v(); }
CView genc(const xrt_unet* n, int l) { return l == n->L - 1 ? n->gebot.cv() : n->gcat[l].cv(); }
View genc_w(xrt_unet* n, int l) { return l == n->L - 1 ? n->gebot.v() : n->gcat[l].v(); }
// output of decoder level l (l == L-1: the bottleneck)
CView dec_out(const xrt_unet* n, int l) { return l == n->L - 1 ? n->ebot.cv() : n->dd[l].cv(); }

hipError_t conv(xrt_unet* n, CView x, const uint16_t* w, View y, CView mask, int B, int H, int W, int cin, int cout,
                bool relu, hipStream_t s, int in_mode = xrl::kConvPlain, CView x2 = CView{nullptr, 0})
{
    xrl::ConvArgs a;
    a.x = x;
    a.in_mode = in_mode;
    a.x2 = x2;
    a.w = w;
    a.y = y.p;
    a.ypitch = y.pitch;
    a.mask = mask;
    a.B = B;
    a.H = H;
    a.W = W;
    a.cin = cin;
    a.cout = cout;
    a.relu = relu ? 1 : 0;
    return xrl::conv3x3(a, false, n->cws, n->cws_n, s);
}

hipError_t wgrad(xrt_unet* n, int k, CView x, CView g, int B, int H, int W, hipStream_t s)
{
    const Layer& Ly = n->layers[k];
    xrl::WgradArgs a;
    a.x = x;
    a.g = g;
    a.part = n->part;
    a.B = B;
    a.H = H;
    a.W = W;
    a.cin = Ly.cin;
    a.cout = Ly.cout;
    a.rows = xrl::wgrad_rows(B, H, W, Ly.cin, Ly.cout);
    int nreg = 0;
    hipError_t e = xrl::conv3x3_wgrad(a, &nreg, s);
    if (e != hipSuccess) return e;
    return xrl::reduce_parts(n->part, nreg, Ly.size(), n->grad + Ly.off, s);
}

hipError_t repack(xrt_unet* n, hipStream_t s)
{
    for (size_t k = 0; k < n->layers.size(); ++k) {
        const Layer& Ly = n->layers[k];
        const bool mfma = Ly.taps == 9 && Ly.cin % 32 == 0;
        hipError_t e = xrl::pack_weights(n->param + Ly.off, Ly.taps, Ly.cout, Ly.cin, n->wf + Ly.woff,
                                         mfma ? n->wb + Ly.woff : nullptr, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// network forward for B images r [B][H][W]; leaves y (normalised output) and all activations.
// With z != nullptr (an apply: no backward follows) the output is unscaled into z instead of
// y, and with n->fuse the pooled encoder inputs and the upsampled halves of the decoder's
// concatenations are read inside the convolutions that consume them (same values, fewer
// launches) and not written out.
hipError_t forward(xrt_unet* n, const float* r, const float* e, int B, hipStream_t s, float* z = nullptr)
{
    const bool fuse = z && n->fuse;
    const int L = n->L;
    const int64_t npix = (int64_t)n->H * n->W;
    const CView none{nullptr, 0};
    hipError_t err;
#define XL_RUN(call)                          \
    do {                                      \
        if ((err = (call)) != hipSuccess) return err; \
    } while (0)
    XL_RUN(xrl::image_stats(r, e, B, npix, n->gain, n->scale, e ? n->tn : nullptr, n->ipart, s));
    // encoder
    for (int l = 0; l < L; ++l) {
        const int H = n->H >> l, W = n->W >> l, c = n->ch[l];
        if (l == 0) {
            XL_RUN(xrl::conv_in(r, n->scale, WF(n, enc_a(n, 0)), n->eh[0].v(), c, B, H, W, n->relu, s));
        } else if (fuse) {
            XL_RUN(conv(n, enc_out(n, l - 1), WF(n, enc_a(n, l)), n->eh[l].v(), none, B, H, W, n->ch[l - 1], c,
                        n->relu, s, xrl::kConvPool));
        } else {
            XL_RUN(xrl::avgpool2(enc_out(n, l - 1), n->in[l].v(), n->ch[l - 1], B, H * 2, W * 2, s));
            XL_RUN(conv(n, n->in[l].cv(), WF(n, enc_a(n, l)), n->eh[l].v(), none, B, H, W, n->ch[l - 1], c, n->relu, s));
        }
        XL_RUN(conv(n, n->eh[l].cv(), WF(n, enc_b(n, l)), enc_out_w(n, l), none, B, H, W, c, c, n->relu, s));
    }
    // decoder
    for (int l = L - 2; l >= 0; --l) {
        const int H = n->H >> l, W = n->W >> l, c = n->ch[l];
        XL_RUN(conv(n, dec_out(n, l + 1), WF(n, dec_up(n, l)), n->uc[l].v(), none, B, H / 2, W / 2, n->ch[l + 1], c,
                    n->relu, s));
        if (fuse) {
            XL_RUN(conv(n, n->cat[l].cv(), WF(n, dec_a(n, l)), n->dh[l].v(), none, B, H, W, 2 * c, c, n->relu, s,
                        xrl::kConvUpcat, n->uc[l].cv()));
        } else {
            XL_RUN(xrl::upsample2(n->uc[l].cv(), n->cat[l].v(c), c, B, H, W, s));
            XL_RUN(conv(n, n->cat[l].cv(), WF(n, dec_a(n, l)), n->dh[l].v(), none, B, H, W, 2 * c, c, n->relu, s));
        }
        XL_RUN(conv(n, n->dh[l].cv(), WF(n, dec_b(n, l)), n->dd[l].v(), none, B, H, W, c, c, n->relu, s));
    }
    if (fuse)
        XL_RUN(xrl::conv_out(n->dd[0].cv(), WF(n, out_layer(n)), n->ch[0], z, (int)(B * npix), s, n->scale, n->gain,
                             npix));
    else
        XL_RUN(xrl::conv_out(n->dd[0].cv(), WF(n, out_layer(n)), n->ch[0], n->y, (int)(B * npix), s));
    if (z && !fuse) XL_RUN(xrl::unscale(n->y, n->scale, B, npix, n->gain, z, s));
    return hipSuccess;
}

// gradient of the loss (gy already in n->gy) w.r.t. every parameter, into n->grad
hipError_t backward(xrt_unet* n, const float* r, int B, hipStream_t s)
{
    const int L = n->L;
    // activation masks apply only with ReLU
    auto MK = [n](CView v) { return n->relu ? v : CView{nullptr, 0}; };
    const int64_t npix = (int64_t)n->H * n->W;
    hipError_t err;
    int nreg = 0;
    {
        const Layer& Lo = n->layers[out_layer(n)];
        XL_RUN(xrl::conv_out_wgrad(n->dd[0].cv(), n->gy, n->ch[0], (int)(B * npix), n->part, &nreg, s));
        XL_RUN(xrl::reduce_parts(n->part, nreg, Lo.size(), n->grad + Lo.off, s));
        XL_RUN(xrl::conv_out_bwd(n->dd[0].cv(), WF(n, out_layer(n)), n->gy, n->ch[0], n->gdd[0].v(),
                                 (int)(B * npix), n->relu, s));
    }
    // decoder, fine to coarse; gdd[l] is the (masked) gradient of decoder level l's output
    for (int l = 0; l <= L - 2; ++l) {
        const int H = n->H >> l, W = n->W >> l, c = n->ch[l];
        XL_RUN(wgrad(n, dec_b(n, l), n->dh[l].cv(), n->gdd[l].cv(), B, H, W, s));
        XL_RUN(conv(n, n->gdd[l].cv(), WB(n, dec_b(n, l)), n->gdh[l].v(), MK(n->dh[l].cv()), B, H, W, c, c, false, s));
        XL_RUN(wgrad(n, dec_a(n, l), n->cat[l].cv(), n->gdh[l].cv(), B, H, W, s));
        XL_RUN(conv(n, n->gdh[l].cv(), WB(n, dec_a(n, l)), n->gcat[l].v(), MK(n->cat[l].cv()), B, H, W, c, 2 * c, false,
                    s));
        XL_RUN(xrl::upsample2_T(n->gcat[l].cv(c), n->guc[l].v(), c, B, H, W, s));
        XL_RUN(wgrad(n, dec_up(n, l), dec_out(n, l + 1), n->guc[l].cv(), B, H / 2, W / 2, s));
        const View tgt = (l + 1 == L - 1) ? n->gebot.v() : n->gdd[l + 1].v();
        XL_RUN(conv(n, n->guc[l].cv(), WB(n, dec_up(n, l)), tgt, MK(dec_out(n, l + 1)), B, H / 2, W / 2, c, n->ch[l + 1],
                    false, s));
    }
    // encoder, coarse to fine; genc(l) holds the masked gradient of encoder level l's output
    for (int l = L - 1; l >= 0; --l) {
        const int H = n->H >> l, W = n->W >> l, c = n->ch[l];
        XL_RUN(wgrad(n, enc_b(n, l), n->eh[l].cv(), genc(n, l), B, H, W, s));
        XL_RUN(conv(n, genc(n, l), WB(n, enc_b(n, l)), n->geh[l].v(), MK(n->eh[l].cv()), B, H, W, c, c, false, s));
        if (l > 0) {
            const int cp = n->ch[l - 1];
            XL_RUN(wgrad(n, enc_a(n, l), n->in[l].cv(), n->geh[l].cv(), B, H, W, s));
            XL_RUN(conv(n, n->geh[l].cv(), WB(n, enc_a(n, l)), n->gin[l].v(), CView{nullptr, 0}, B, H, W, c, cp, false,
                        s));
            XL_RUN(xrl::avgpool2_T_add(n->gin[l].cv(), genc_w(n, l - 1), MK(enc_out(n, l - 1)), cp, B, 2 * H, 2 * W, s));
        } else {
            const Layer& La = n->layers[enc_a(n, 0)];
            XL_RUN(xrl::conv_in_wgrad(r, n->scale, n->geh[0].cv(), c, B, H, W, n->part, &nreg, s));
            XL_RUN(xrl::reduce_parts(n->part, nreg, La.size(), n->grad + La.off, s));
        }
    }
    return hipSuccess;
}

// one Adam step on the master parameters from n->grad, then the bf16 copies
xrt_status adam_update(xrt_unet* n, float lr, hipStream_t s)
{
    n->step += 1;
    const double b1 = 0.9, b2 = 0.999;
    const float c1 = (float)(1.0 / (1.0 - pow(b1, (double)n->step)));
    const float c2 = (float)(1.0 / (1.0 - pow(b2, (double)n->step)));
    XL_CHECK(xrl::adam(n->param, n->grad, n->m, n->v, n->nparam, lr, (float)b1, (float)b2, 1e-8f, c1, c2, s), "adam");
    XL_CHECK(repack(n, s), "pack_weights");
    return XRT_OK;
}

void free_all(xrt_unet* n)
{
    for (void* p : n->allocs) (void)hipFree(p);
    n->allocs.clear();
}

}  // namespace

extern "C" {

xrt_status xrt_reg_apply(const float* c, int32_t nx, int32_t ny, float lambda, float* out, void* stream)
{
    if (!c || !out || nx < 1 || ny < 1) return XRT_EINVAL;
    XL_CHECK(xrl::reg_apply(c, out, nx, ny, lambda, false, (hipStream_t)stream), "reg_apply");
    return XRT_OK;
}

xrt_status xrt_normal_apply(const xrt_plan* plan, float lambda, const float* c, float* out, float* sino_ws,
                            void* stream)
{
    if (!c || !out) return XRT_EINVAL;
    int64_t m = 0, crossing = 0;
    xrt_status st = xrt_plan_info(plan, &m, &crossing);
    if (st != XRT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    float* sino = sino_ws;
    if (!sino) XL_CHECK(hipMallocAsync((void**)&sino, (size_t)(m > 0 ? m : 1) * sizeof(float), s), "hipMallocAsync");
    st = xrt_plan_forward(plan, c, sino, stream);
    if (st == XRT_OK) st = xrt_plan_adjoint(plan, sino, out, stream);
    if (st == XRT_OK) {
        hipError_t e = xrl::reg_apply(c, out, plan->g.nx, plan->g.ny, lambda, true, s);
        if (e != hipSuccess) st = hip_fail("reg_apply", e);
    }
    if (!sino_ws) (void)hipFreeAsync(sino, s);
    return st;
}

xrt_status xrt_unet_create(int32_t levels, int32_t base, int32_t max_channels, int32_t height, int32_t width,
                           int32_t max_batch, uint64_t seed, xrt_unet** out)
{
    if (!out) return XRT_EINVAL;
    *out = nullptr;
    if (levels < 2 || levels > 8 || base < 32 || base % 32 || 256 % base || max_channels < 0 || max_channels % 32)
        return XRT_EINVAL;
    const int cap = max_channels > 0 ? max_channels : 512;
    if (cap < base || cap > 512) return XRT_EINVAL;
    const int mult = 1 << (levels - 1);
    if (height < mult || width < mult || height % mult || width % mult || max_batch < 1) return XRT_ESIZE;
    if ((int64_t)height * width * max_batch > (int64_t)1 << 28 || max_batch > 65535) return XRT_ESIZE;

    xrt_unet* n = new xrt_unet();
    n->magic = kNetMagic;
    n->L = levels;
    n->base = base;
    n->H = height;
    n->W = width;
    n->maxB = max_batch;
    n->step = 0;
    n->gain = 1.f;
    n->relu = true;
    for (int l = 0; l < levels; ++l) n->ch[l] = std::min(base << l, cap);
    // parameter layout (the order documented in xrt_learn.h)
    auto add = [&](int taps, int cout, int cin) {
        Layer Ly;
        Ly.taps = taps;
        Ly.cout = cout;
        Ly.cin = cin;
        Ly.off = n->layers.empty() ? 0 : n->layers.back().off + n->layers.back().size();
        Ly.woff = n->layers.empty() ? 0
                                    : (n->layers.back().woff + n->layers.back().size() + 63) / 64 * 64;
        n->layers.push_back(Ly);
    };
    for (int l = 0; l < levels; ++l) {
        add(9, n->ch[l], l == 0 ? 1 : n->ch[l - 1]);
        add(9, n->ch[l], n->ch[l]);
    }
    for (int l = levels - 2; l >= 0; --l) {
        add(9, n->ch[l], n->ch[l + 1]);
        add(9, n->ch[l], 2 * n->ch[l]);
        add(9, n->ch[l], n->ch[l]);
    }
    add(1, 1, n->ch[0]);   // out: [c_0] (one tap, one output, c_0 inputs)
    n->nparam = n->layers.back().off + n->layers.back().size();
    n->nw = n->layers.back().woff + n->layers.back().size() + 64;

    // workspace sizes
    int64_t part_n = 0;
    const int B = max_batch;
    for (size_t k = 0; k < n->layers.size(); ++k) {
        const Layer& Ly = n->layers[k];
        // level of the layer's output / wgrad pixel grid
        int lev = 0;
        if ((int)k < 2 * levels) lev = (int)k / 2;
        else if ((int)k < out_layer(n)) {
            const int j = ((int)k - 2 * levels) / 3, kind = ((int)k - 2 * levels) % 3;
            const int l = levels - 2 - j;
            lev = kind == 0 ? l + 1 : l;
        }
        const int H = height >> lev, W = width >> lev;
        int64_t need;
        if (Ly.taps == 9 && Ly.cin % 32 == 0) {
            const int rows = xrl::wgrad_rows(B, H, W, Ly.cin, Ly.cout);
            need = xrl::wgrad_regions(B, H, W, rows) * Ly.size();
        } else {
            const int64_t np = (int64_t)B * H * W;
            const int64_t per = xrl::per_block_pixels(np);
            need = (np + per - 1) / per * 9 * n->ch[0];
        }
        if (need > part_n) part_n = need;
    }
    n->part_n = part_n;
    int64_t cws_n = 0;
    for (size_t k = 0; k < n->layers.size(); ++k) {
        const Layer& Ly = n->layers[k];
        if (!(Ly.taps == 9 && Ly.cin % 32 == 0)) continue;
        // the split depends on the batch actually passed (<= max_batch)
        for (int lev = 0; lev < levels; ++lev)
            for (int b = 1; b <= std::min(B, 64); ++b) {
                const int H = height >> lev, W = width >> lev;
                cws_n = std::max(cws_n, xrl::conv3x3_ws_floats(b, H, W, Ly.cin, Ly.cout));
                cws_n = std::max(cws_n, xrl::conv3x3_ws_floats(b, H, W, Ly.cout, Ly.cin));
            }
    }
    n->cws_n = cws_n;

    bool ok = true;
    auto alloc = [&](size_t bytes) -> void* {
        void* p = nullptr;
        if (!ok) return nullptr;
        if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
            ok = false;
            return nullptr;
        }
        n->allocs.push_back(p);
        return p;
    };
    auto buf = [&](int lev, int c) {
        Buf b;
        b.c = c;
        b.p = (uint16_t*)alloc((size_t)B * (height >> lev) * (width >> lev) * c * sizeof(uint16_t));
        return b;
    };
    n->param = (float*)alloc(n->nparam * sizeof(float));
    n->grad = (float*)alloc(n->nparam * sizeof(float));
    n->m = (float*)alloc(n->nparam * sizeof(float));
    n->v = (float*)alloc(n->nparam * sizeof(float));
    n->wf = (uint16_t*)alloc(n->nw * sizeof(uint16_t));
    n->wb = (uint16_t*)alloc(n->nw * sizeof(uint16_t));
    for (int l = 0; l < levels; ++l) {
        const int c = n->ch[l];
        if (l > 0) {
            n->in[l] = buf(l, n->ch[l - 1]);
            n->gin[l] = buf(l, n->ch[l - 1]);
        }
        n->eh[l] = buf(l, c);
        n->geh[l] = buf(l, c);
        if (l < levels - 1) {
            n->cat[l] = buf(l, 2 * c);
            n->gcat[l] = buf(l, 2 * c);
            n->uc[l] = buf(l + 1, c);
            n->guc[l] = buf(l + 1, c);
            n->dh[l] = buf(l, c);
            n->gdh[l] = buf(l, c);
            n->dd[l] = buf(l, c);
            n->gdd[l] = buf(l, c);
        } else {
            n->ebot = buf(l, c);
            n->gebot = buf(l, c);
        }
    }
    const int64_t npix = (int64_t)B * height * width;
    n->scale = (float*)alloc(B * sizeof(float));
    n->tn = (float*)alloc(B * sizeof(float));
    n->y = (float*)alloc(npix * sizeof(float));
    n->gy = (float*)alloc(npix * sizeof(float));
    n->lpart = (float*)alloc(256 * sizeof(float));
    n->loss_tmp = (float*)alloc(sizeof(float));
    n->part = (float*)alloc(part_n * sizeof(float));
    n->ipart = (double*)alloc((size_t)xrl::image_parts() * 2 * B * sizeof(double));
    n->cws = n->cws_n > 0 ? (float*)alloc(n->cws_n * sizeof(float)) : nullptr;
    if (!ok) {
        free_all(n);
        delete n;
        return XRT_ENOMEM;
    }
    // He-normal initialisation on the host (deterministic for a seed)
    std::vector<float> h(n->nparam);
    std::mt19937_64 rng(seed);
    for (size_t k = 0; k < n->layers.size(); ++k) {
        const Layer& Ly = n->layers[k];
        const bool last = (int)k == out_layer(n);
        const double sd = last ? sqrt(1.0 / Ly.cin) : sqrt(2.0 / (Ly.taps * Ly.cin));
        std::normal_distribution<double> nd(0.0, sd);
        for (int64_t i = 0; i < Ly.size(); ++i) h[Ly.off + i] = (float)nd(rng);
    }
    hipError_t e = hipMemcpy(n->param, h.data(), n->nparam * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(n->m, 0, n->nparam * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->v, 0, n->nparam * sizeof(float));
    if (e == hipSuccess) e = hipMemset(n->wf, 0, n->nw * sizeof(uint16_t));
    if (e == hipSuccess) e = hipMemset(n->wb, 0, n->nw * sizeof(uint16_t));
    if (e == hipSuccess) e = repack(n, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        free_all(n);
        delete n;
        return hip_fail("xrt_unet_create", e);
    }
    *out = n;
    return XRT_OK;
}

void xrt_unet_destroy(xrt_unet* net)
{
    if (!net_ok(net)) return;
    (void)hipDeviceSynchronize();
    free_all(net);
    net->magic = 0;
    delete net;
}

xrt_status xrt_unet_num_params(const xrt_unet* net, int64_t* n)
{
    if (!net_ok(net) || !n) return XRT_EINVAL;
    *n = net->nparam;
    return XRT_OK;
}

xrt_status xrt_unet_set_params(xrt_unet* net, const float* params, void* stream)
{
    if (!net_ok(net) || !params) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    XL_CHECK(hipMemcpyAsync(net->param, params, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, s),
             "hipMemcpyAsync");
    XL_CHECK(xrl::fill_f32(net->m, net->nparam, 0.f, s), "fill");
    XL_CHECK(xrl::fill_f32(net->v, net->nparam, 0.f, s), "fill");
    net->step = 0;
    XL_CHECK(repack(net, s), "pack_weights");
    return XRT_OK;
}

xrt_status xrt_unet_set_gain(xrt_unet* net, float gain)
{
    if (!net_ok(net) || !(gain > 0.f) || !isfinite(gain)) return XRT_EINVAL;
    net->gain = gain;
    return XRT_OK;
}

xrt_status xrt_unet_set_relu(xrt_unet* net, int32_t on)
{
    if (!net_ok(net)) return XRT_EINVAL;
    net->relu = on != 0;
    return XRT_OK;
}

xrt_status xrt_unet_set_fusion(xrt_unet* net, int32_t on)
{
    if (!net_ok(net) || (on != 0 && on != 1)) return XRT_EINVAL;
    net->fuse = on != 0;
    return XRT_OK;
}

xrt_status xrt_unet_get_gain(const xrt_unet* net, float* gain)
{
    if (!net_ok(net) || !gain) return XRT_EINVAL;
    *gain = net->gain;
    return XRT_OK;
}

xrt_status xrt_unet_get_params(const xrt_unet* net, float* params, void* stream)
{
    if (!net_ok(net) || !params) return XRT_EINVAL;
    XL_CHECK(hipMemcpyAsync(params, net->param, net->nparam * sizeof(float), hipMemcpyDeviceToDevice,
                            (hipStream_t)stream),
             "hipMemcpyAsync");
    return XRT_OK;
}

xrt_status xrt_unet_apply(xrt_unet* net, const float* r, float* z, int32_t batch, void* stream)
{
    if (!net_ok(net) || !r || !z || batch < 1 || batch > net->maxB) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    XL_CHECK(forward(net, r, nullptr, batch, s, z), "unet forward");
    return XRT_OK;
}

xrt_status xrt_unet_loss_grad(xrt_unet* net, const float* r, const float* e, int32_t batch, float* loss,
                              float* grad, void* stream)
{
    if (!net_ok(net) || !r || !e || !loss || batch < 1 || batch > net->maxB) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = (int64_t)net->H * net->W;
    XL_CHECK(forward(net, r, e, batch, s), "unet forward");
    XL_CHECK(xrl::loss_grad(net->y, e, net->scale, net->tn, batch, npix, net->gain, net->gy, net->lpart, loss, s),
             "loss");
    if (grad) {
        XL_CHECK(backward(net, r, batch, s), "unet backward");
        if (grad != net->grad)
            XL_CHECK(hipMemcpyAsync(grad, net->grad, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, s),
                     "hipMemcpyAsync");
    }
    return XRT_OK;
}

xrt_status xrt_unet_train_step(xrt_unet* net, const float* r, const float* e, int32_t batch, float lr, float* loss,
                               void* stream)
{
    if (!net_ok(net) || !r || !e || !loss || batch < 1 || batch > net->maxB || !(lr > 0.f)) return XRT_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    xrt_status st = xrt_unet_loss_grad(net, r, e, batch, loss, net->grad, stream);
    if (st != XRT_OK) return st;
    return adam_update(net, lr, s);
}

xrt_status xrt_unet_loss_grad_normal(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                     int32_t batch, float* loss, float* grad, void* stream)
{
    if (!net_ok(net) || !r || !loss || batch < 1 || batch > net->maxB) return XRT_EINVAL;
    int64_t m = 0, crossing = 0;
    xrt_status st = xrt_plan_info(plan, &m, &crossing);
    if (st != XRT_OK) return st;
    if (plan->g.nx != net->W || plan->g.ny != net->H) return XRT_ESIZE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = (int64_t)net->H * net->W, nb = (int64_t)batch * npix;
    // workspace: z, q (= M z, then M d), d; sinogram; per-image sums
    float* ws = nullptr;
    const int64_t ms = m > 0 ? m : 1;
    XL_CHECK(hipMallocAsync((void**)&ws, (3 * nb + ms + 2 * (int64_t)batch) * sizeof(float), s), "hipMallocAsync");
    float *z = ws, *q = ws + nb, *d = ws + 2 * nb, *sino = ws + 3 * nb;
    float *rr = sino + ms, *lb = rr + batch;
    hipError_t e = forward(net, r, nullptr, batch, s);
    if (e == hipSuccess) e = xrl::unscale(net->y, net->scale, batch, npix, net->gain, z, s);
    for (int b = 0; b < batch && e == hipSuccess && st == XRT_OK; ++b)
        st = xrt_normal_apply(plan, lambda, z + b * npix, q + b * npix, sino, stream);
    if (e == hipSuccess && st == XRT_OK) e = xrl::resid_stats(q, r, d, batch, npix, rr, lb, loss, net->ipart, s);
    if (grad && e == hipSuccess && st == XRT_OK) {
        for (int b = 0; b < batch && st == XRT_OK; ++b)
            st = xrt_normal_apply(plan, lambda, d + b * npix, q + b * npix, sino, stream);
        if (st == XRT_OK) e = xrl::resid_grad(q, net->scale, rr, batch, npix, net->gain, net->gy, s);
        if (e == hipSuccess && st == XRT_OK) e = backward(net, r, batch, s);
        if (e == hipSuccess && st == XRT_OK && grad != net->grad)
            e = hipMemcpyAsync(grad, net->grad, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    (void)hipFreeAsync(ws, s);
    if (e != hipSuccess) return hip_fail("unet residual loss", e);
    return st;
}

xrt_status xrt_unet_train_step_normal(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                      int32_t batch, float lr, float* loss, void* stream)
{
    if (!(lr > 0.f)) return XRT_EINVAL;
    xrt_status st = xrt_unet_loss_grad_normal(net, plan, lambda, r, batch, loss, net_ok(net) ? net->grad : nullptr,
                                              stream);
    if (st != XRT_OK) return st;
    return adam_update(net, lr, (hipStream_t)stream);
}

xrt_status xrt_unet_loss_grad_energy(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                     const float* e_in, int32_t batch, float* loss, float* grad, void* stream)
{
    if (!net_ok(net) || !r || !e_in || !loss || batch < 1 || batch > net->maxB) return XRT_EINVAL;
    int64_t m = 0, crossing = 0;
    xrt_status st = xrt_plan_info(plan, &m, &crossing);
    if (st != XRT_OK) return st;
    if (plan->g.nx != net->W || plan->g.ny != net->H) return XRT_ESIZE;
    hipStream_t s = (hipStream_t)stream;
    const int64_t npix = (int64_t)net->H * net->W, nb = (int64_t)batch * npix;
    // workspace: z, q (= M z), d (= q - r); sinogram; per-image sums; the
    // per-image partial sums of the three dot products
    float* ws = nullptr;
    const int64_t ms = m > 0 ? m : 1;
    const int64_t parts = 3 * (int64_t)xrl::image_parts() * batch;
    XL_CHECK(hipMallocAsync((void**)&ws, (3 * nb + ms + 2 * (int64_t)batch) * sizeof(float) + parts * sizeof(double),
                            s),
             "hipMallocAsync");
    float *z = ws, *q = ws + nb, *d = ws + 2 * nb, *sino = ws + 3 * nb;
    float *er = sino + ms, *lb = er + batch;
    double* part = (double*)(ws + 3 * nb + ms + 2 * (int64_t)batch);
    hipError_t e = forward(net, r, nullptr, batch, s);
    if (e == hipSuccess) e = xrl::unscale(net->y, net->scale, batch, npix, net->gain, z, s);
    for (int b = 0; b < batch && e == hipSuccess && st == XRT_OK; ++b)
        st = xrt_normal_apply(plan, lambda, z + b * npix, q + b * npix, sino, stream);
    if (e == hipSuccess && st == XRT_OK) e = xrl::energy_stats(z, q, r, e_in, d, batch, npix, er, lb, loss, part, s);
    if (grad && e == hipSuccess && st == XRT_OK) {
        e = xrl::resid_grad(d, net->scale, er, batch, npix, net->gain, net->gy, s);
        if (e == hipSuccess) e = backward(net, r, batch, s);
        if (e == hipSuccess && grad != net->grad)
            e = hipMemcpyAsync(grad, net->grad, net->nparam * sizeof(float), hipMemcpyDeviceToDevice, s);
    }
    (void)hipFreeAsync(ws, s);
    if (e != hipSuccess) return hip_fail("unet energy loss", e);
    return st;
}

xrt_status xrt_unet_train_step_energy(xrt_unet* net, const xrt_plan* plan, float lambda, const float* r,
                                      const float* e, int32_t batch, float lr, float* loss, void* stream)
{
    if (!(lr > 0.f)) return XRT_EINVAL;
    xrt_status st = xrt_unet_loss_grad_energy(net, plan, lambda, r, e, batch, loss,
                                              net_ok(net) ? net->grad : nullptr, stream);
    if (st != XRT_OK) return st;
    return adam_update(net, lr, (hipStream_t)stream);
}

static xrt_status check_conv_args(const void* a, const void* b, int32_t B, int32_t H, int32_t W, int32_t cin,
                                  int32_t cout, const void* out)
{
    if (!a || !b || !out || B < 1 || B > 65535 || H < 1 || W < 1 || cin < 32 || cout < 32 || cin % 32 || cout % 32)
        return XRT_EINVAL;
    return XRT_OK;
}

xrt_status xrt_conv3x3_forward(const uint16_t* x, const uint16_t* w, int32_t B, int32_t H, int32_t W, int32_t cin,
                               int32_t cout, int32_t relu, float* y, void* stream)
{
    xrt_status st = check_conv_args(x, w, B, H, W, cin, cout, y);
    if (st != XRT_OK) return st;
    xrl::ConvArgs a;
    a.x = CView{x, cin};
    a.w = w;
    a.y = y;
    a.ypitch = cout;
    a.mask = CView{nullptr, 0};
    a.B = B;
    a.H = H;
    a.W = W;
    a.cin = cin;
    a.cout = cout;
    a.relu = relu ? 1 : 0;
    hipStream_t s = (hipStream_t)stream;
    const int64_t wn = xrl::conv3x3_ws_floats(B, H, W, cin, cout);
    float* ws = nullptr;
    if (wn > 0) XL_CHECK(hipMallocAsync((void**)&ws, wn * sizeof(float), s), "hipMallocAsync");
    hipError_t e = xrl::conv3x3(a, true, ws, wn, s);
    if (ws) (void)hipFreeAsync(ws, s);
    XL_CHECK(e, "conv3x3");
    return XRT_OK;
}

xrt_status xrt_conv3x3_grad_input(const uint16_t* gy, const uint16_t* w, int32_t B, int32_t H, int32_t W,
                                  int32_t cin, int32_t cout, float* gx, void* stream)
{
    xrt_status st = check_conv_args(gy, w, B, H, W, cin, cout, gx);
    if (st != XRT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t nw = (int64_t)9 * cout * cin;
    Scratch tmp(s);
    uint16_t* wflip = nullptr;
    XL_CHECK(tmp.device(&wflip, nw * sizeof(uint16_t)), "hipMallocAsync");
    XL_CHECK(xrl::flip_weights(w, 9, cout, cin, wflip, s), "flip_weights");
    xrl::ConvArgs a;
    a.x = CView{gy, cout};
    a.w = wflip;
    a.y = gx;
    a.ypitch = cin;
    a.mask = CView{nullptr, 0};
    a.B = B;
    a.H = H;
    a.W = W;
    a.cin = cout;
    a.cout = cin;
    a.relu = 0;
    const int64_t wn = xrl::conv3x3_ws_floats(B, H, W, cout, cin);
    float* ws = nullptr;
    if (wn > 0) XL_CHECK(tmp.device(&ws, wn * sizeof(float)), "hipMallocAsync");
    XL_CHECK(xrl::conv3x3(a, true, ws, wn, s), "conv3x3");
    return XRT_OK;
}

xrt_status xrt_conv3x3_grad_weight(const uint16_t* x, const uint16_t* gy, int32_t B, int32_t H, int32_t W,
                                   int32_t cin, int32_t cout, float* gw, void* stream)
{
    xrt_status st = check_conv_args(x, gy, B, H, W, cin, cout, gw);
    if (st != XRT_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    xrl::WgradArgs a;
    a.x = CView{x, cin};
    a.g = CView{gy, cout};
    a.B = B;
    a.H = H;
    a.W = W;
    a.cin = cin;
    a.cout = cout;
    a.rows = xrl::wgrad_rows(B, H, W, cin, cout);
    const int64_t nreg = xrl::wgrad_regions(B, H, W, a.rows);
    Scratch tmp(s);
    XL_CHECK(tmp.device(&a.part, (size_t)nreg * 9 * cin * cout * sizeof(float)), "hipMallocAsync");
    int nr = 0;
    XL_CHECK(xrl::conv3x3_wgrad(a, &nr, s), "conv3x3_wgrad");
    XL_CHECK(xrl::reduce_parts(a.part, nr, (int64_t)9 * cin * cout, gw, s), "reduce");
    return XRT_OK;
}

// ------------------------------------------------------------------ solvers
// device scalar slots; S_RP must follow S_PQ (pair of dots); S_ZQ and S_PQR hold one
// entry per stored direction
enum { S_RR = 0, S_PQ, S_RP, S_RRN, S_BB, S_ZQ = 8, S_PQR = S_ZQ + xrl::kMaxVecs, S_N = S_PQR + xrl::kMaxVecs };

xrt_status xrt_solve(const xrt_plan* plan, float lambda, const float* b, float* x, float tol, int32_t maxit,
                     xrt_unet* net, int32_t window, int32_t period, xrt_solve_info* info, double* history,
                     int32_t history_cap, void* stream)
{
    xrt_solve_opts o;
    o.window = window;
    o.period = period;
    o.net_steps = 0;
    o.restart = 0;
    return xrt_solve_ex(plan, lambda, b, x, tol, maxit, net, net ? &o : nullptr, info, history, history_cap,
                        stream);
}

xrt_status xrt_solve_ex(const xrt_plan* plan, float lambda, const float* b, float* x, float tol, int32_t maxit,
                        xrt_unet* net, const xrt_solve_opts* opts, xrt_solve_info* info, double* history,
                        int32_t history_cap, void* stream)
{
    if (!b || !x || !info || !(tol > 0.f) || maxit < 0) return XRT_EINVAL;
    if (net && !opts) return XRT_EINVAL;
    const int32_t window = net ? opts->window : 1, period = net ? opts->period : 1;
    const int32_t net_steps = net ? opts->net_steps : 0;
    const bool restart = net && opts->restart != 0;
    if (net && (window < 1 || window > xrl::kMaxVecs || period < 1 || net_steps < 0)) return XRT_EINVAL;
    if (net && (opts->restart != 0 && opts->restart != 1)) return XRT_EINVAL;
    if (restart && net_steps == 0) return XRT_EINVAL;
    int64_t m = 0, crossing = 0;
    xrt_status st = xrt_plan_info(plan, &m, &crossing);
    if (st != XRT_OK) return st;
    if (net && !net_ok(net)) return XRT_EINVAL;
    const int nx = plan->g.nx, ny = plan->g.ny;
    if (net && (net->H != ny || net->W != nx)) return XRT_ESIZE;
    memset(info, 0, sizeof(*info));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)nx * ny;
    const int win = net ? window : 0;

    // workspace: r, r_new, x_new, p_new, q, z, p (CG), then 2*win ring vectors; one sinogram; scalars
    const int nvec = 7 + 2 * win;
    Scratch tmp(s);
    float* ws = nullptr;
    double *slots = nullptr, *dpart = nullptr, *host = nullptr;
    XL_CHECK(tmp.device(&ws, ((size_t)nvec * n + (size_t)(m > 0 ? m : 1)) * sizeof(float)), "hipMallocAsync");
    XL_CHECK(tmp.device(&slots, S_N * sizeof(double)), "hipMallocAsync");
    XL_CHECK(tmp.device(&dpart, (size_t)xrl::kMaxVecs * xrl::dots_parts() * sizeof(double)), "hipMallocAsync");
    XL_CHECK(tmp.host(&host, S_N * sizeof(double)), "hipHostMalloc");
    float *r = ws, *rn = ws + n, *xn = ws + 2 * n, *pn = ws + 3 * n, *q = ws + 4 * n, *z = ws + 5 * n,
          *p = ws + 6 * n, *sino = ws + (size_t)nvec * n;
    float* P[xrl::kMaxVecs];
    float* Q[xrl::kMaxVecs];
    for (int k = 0; k < win; ++k) {
        P[k] = ws + (size_t)(7 + 2 * k) * n;
        Q[k] = ws + (size_t)(8 + 2 * k) * n;
    }
    int cnt = 0, head = 0;      // stored directions, oldest entry once full
    float* xc = x;              // current iterate (x or xn)

    hipError_t e = hipSuccess;
    auto M = [&](const float* in, float* outv) -> xrt_status {
        info->operator_applies += 1;
        return xrt_normal_apply(plan, lambda, in, outv, sino, stream);
    };
    auto read_slots = [&]() -> hipError_t {
        hipError_t er = hipMemcpyAsync(host, slots, S_N * sizeof(double), hipMemcpyDeviceToHost, s);
        if (er == hipSuccess) er = hipStreamSynchronize(s);
        return er;
    };
#define XS(call, what)                                  \
    do {                                                \
        if ((e = (call)) != hipSuccess) {               \
            st = hip_fail(what, e);                     \
            goto done;                                  \
        }                                               \
    } while (0)
#define XM(call)                                        \
    do {                                                \
        if ((st = (call)) != XRT_OK) goto done;         \
    } while (0)

    {
        double bn = 0.0, rel = 1.0;
        int hist_n = 0;
        bool have_prev = false, confirmed = false;
        XS(xrl::fill_f32(xc, n, 0.f, s), "fill");
        XS(hipMemcpyAsync(r, b, n * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        XS(xrl::dots(n, b, b, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_BB, s), "dots");
        XS(xrl::copy_slot(slots, S_RR, S_BB, s), "copy");
        XS(read_slots(), "sync");
        bn = sqrt(host[S_BB]);
        if (bn == 0.0) {
            info->converged = 1;
            goto done;
        }
        while (true) {
            if (rel <= tol) {
                // confirm with the explicitly computed residual r = b - M x
                XM(M(xc, q));
                XS(xrl::axpy2(n, slots, S_BB, S_BB, -1, b, q, r, nullptr, nullptr, nullptr, s), "axpy");
                XS(xrl::dots(n, r, r, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_RR, s), "dots");
                XS(read_slots(), "sync");
                rel = sqrt(host[S_RR]) / bn;
                if (rel <= tol) {
                    confirmed = true;
                    break;
                }
                have_prev = false;   // restart from the true residual
                cnt = head = 0;
            }
            if (info->iterations >= maxit) break;
            // with `restart`, the steps after the first net_steps are plain CG, started
            // afresh from the current iterate and residual
            const bool cg_step = !net || (restart && info->iterations >= net_steps);
            if (restart && info->iterations == net_steps) have_prev = false;
            if (cg_step) {
                // conjugate gradients (Hestenes-Stiefel)
                if (!have_prev) {
                    XS(hipMemcpyAsync(p, r, n * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
                    have_prev = true;
                }
                XM(M(p, q));
                XS(xrl::dots(n, p, q, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_PQ, s), "dots");
                XS(xrl::axpy2(n, slots, S_RR, S_PQ, 1, xc, p, xc, r, q, r, s), "axpy");
                XS(xrl::dots(n, r, r, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_RRN, s), "dots");
                XS(xrl::direction(n, slots, S_RRN, -1, S_RR, r, p, p, s), "direction");
                XS(xrl::copy_slot(slots, S_RR, S_RRN, s), "copy");
                XS(read_slots(), "sync");
                rel = sqrt(host[S_RR]) / bn;
            } else {
                // flexible CG: the new direction is M-orthogonalised against the last `win` ones;
                // the network proposes every `period`-th step (within the first net_steps
                // steps when net_steps > 0), the others take z = r
                bool learned = info->iterations % period == 0 && (net_steps == 0 || info->iterations < net_steps);
                for (;;) {
                    const float* zz = r;
                    if (learned) {
                        XM(xrt_unet_apply(net, r, z, 1, stream));
                        zz = z;
                    }
                    xrl::VecList Ql{}, Pl{};
                    for (int k = 0; k < cnt; ++k) {
                        Ql.v[k] = Q[k];
                        Pl.v[k] = P[k];
                    }
                    if (cnt > 0) XS(xrl::dots_multi(n, zz, Ql, cnt, dpart, slots, S_ZQ, s), "dots");
                    XS(xrl::orth(n, slots, S_ZQ, S_PQR, cnt, zz, Pl, pn, s), "orth");
                    XM(M(pn, q));
                    // alpha = <r, p> / <p, M p>; x_new = x + alpha p; r_new = r - alpha M p
                    XS(xrl::dots(n, pn, q, r, pn, nullptr, nullptr, dpart, slots, S_PQ, s), "dots");
                    XS(xrl::axpy2(n, slots, S_RP, S_PQ, 1, xc, pn, xn, r, q, rn, s), "axpy");
                    XS(xrl::dots(n, rn, rn, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_RRN, s), "dots");
                    XS(read_slots(), "sync");
                    if (learned && !(host[S_RRN] < host[S_RR])) {
                        info->learned_rejected += 1;
                        learned = false;
                        continue;
                    }
                    if (learned) info->learned_accepted += 1;
                    break;
                }
                // accept: rotate buffers and store (p, M p) in the window
                float* t;
                t = r; r = rn; rn = t;
                t = xc; xc = xn; xn = t;
                int slot;
                if (cnt < win) slot = cnt++;
                else {
                    slot = head;
                    head = (head + 1) % win;
                }
                t = P[slot]; P[slot] = pn; pn = t;
                t = Q[slot]; Q[slot] = q; q = t;
                XS(xrl::copy_slot(slots, S_PQR + slot, S_PQ, s), "copy");
                XS(xrl::copy_slot(slots, S_RR, S_RRN, s), "copy");
                host[S_RR] = host[S_RRN];
                rel = sqrt(host[S_RR]) / bn;
            }
            info->iterations += 1;
            if (history && hist_n < history_cap) history[hist_n++] = rel;
        }
        if (!confirmed) {
            // report the true residual of the final iterate
            XM(M(xc, q));
            XS(xrl::axpy2(n, slots, S_BB, S_BB, -1, b, q, r, nullptr, nullptr, nullptr, s), "axpy");
            XS(xrl::dots(n, r, r, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_RR, s), "dots");
            XS(read_slots(), "sync");
            rel = sqrt(host[S_RR]) / bn;
        }
        if (xc != x) XS(hipMemcpyAsync(x, xc, n * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        info->rel_residual = rel;
        info->converged = rel <= tol ? 1 : 0;
    }
done:
    (void)hipStreamSynchronize(s);
    return st;
}

static bool filter_ok(int32_t taps) { return taps >= 1 && taps <= 63 && taps % 2 == 1; }

xrt_status xrt_sino_filter(const float* sino, int64_t n_views, int32_t n_bins, const float* filter, int32_t taps,
                           float* out, void* stream)
{
    if (!sino || !filter || !out || n_views < 0 || n_bins < 1 || !filter_ok(taps)) return XRT_EINVAL;
    XL_CHECK(xrl::sino_filter(sino, n_views, n_bins, filter, taps, out, (hipStream_t)stream), "sino_filter");
    return XRT_OK;
}

// slots of the preconditioned CG (the S_* slots 5..7 are free in xrt_solve_ex's layout)
enum { T_RZ = 5, T_RZN = 6, T_RRN = 7 };

xrt_status xrt_solve_sino_pcg(const xrt_plan* plan, float lambda, const float* b, float* x, float tol,
                              int32_t maxit, const xrt_sino_precond* pc, xrt_solve_info* info, double* history,
                              int32_t history_cap, void* stream)
{
    int64_t m = 0, crossing = 0;
    xrt_status st = xrt_plan_info(plan, &m, &crossing);
    if (st != XRT_OK) return st;
    if (!b || !x || !info || !pc || !pc->filter || !(tol > 0.f) || maxit < 0) return XRT_EINVAL;
    if (!filter_ok(pc->taps) || !(pc->mu >= 0.f) || !isfinite(pc->mu)) return XRT_EINVAL;
    if (pc->n_views < 0 || pc->n_bins < 1 || pc->n_views * (int64_t)pc->n_bins != m) return XRT_EINVAL;
    memset(info, 0, sizeof(*info));
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = (int64_t)plan->g.nx * plan->g.ny;
    const int64_t ms = m > 0 ? m : 1;

    // workspace: r, z, p, q; two sinograms; scalars
    Scratch tmp(s);
    float* ws = nullptr;
    double *slots = nullptr, *dpart = nullptr, *host = nullptr;
    XL_CHECK(tmp.device(&ws, ((size_t)4 * n + 2 * (size_t)ms) * sizeof(float)), "hipMallocAsync");
    XL_CHECK(tmp.device(&slots, S_N * sizeof(double)), "hipMallocAsync");
    XL_CHECK(tmp.device(&dpart, (size_t)xrl::kMaxVecs * xrl::dots_parts() * sizeof(double)), "hipMallocAsync");
    XL_CHECK(tmp.host(&host, S_N * sizeof(double)), "hipHostMalloc");
    float *r = ws, *z = ws + n, *p = ws + 2 * n, *q = ws + 3 * n, *sa = ws + 4 * n, *sb = sa + ms;

    hipError_t e = hipSuccess;
    auto M = [&](const float* in, float* outv) -> xrt_status {
        info->operator_applies += 1;
        return xrt_normal_apply(plan, lambda, in, outv, sa, stream);
    };
    // z = H^T (f * (H r)) + mu r
    auto P = [&](const float* in, float* outv) -> xrt_status {
        info->learned_accepted += 1;
        xrt_status t = xrt_plan_forward(plan, in, sa, stream);
        if (t != XRT_OK) return t;
        hipError_t er = xrl::sino_filter(sa, pc->n_views, pc->n_bins, pc->filter, pc->taps, sb, s);
        if (er != hipSuccess) return hip_fail("sino_filter", er);
        t = xrt_plan_adjoint(plan, sb, outv, stream);
        if (t != XRT_OK) return t;
        if (pc->mu > 0.f) {
            er = xrl::add_scaled(n, pc->mu, in, outv, s);
            if (er != hipSuccess) return hip_fail("add_scaled", er);
        }
        return XRT_OK;
    };
    auto read_slots = [&]() -> hipError_t {
        hipError_t er = hipMemcpyAsync(host, slots, S_N * sizeof(double), hipMemcpyDeviceToHost, s);
        if (er == hipSuccess) er = hipStreamSynchronize(s);
        return er;
    };
    {
        double bn = 0.0, rel = 1.0;
        int hist_n = 0;
        bool fresh = true, confirmed = false;
        XS(xrl::fill_f32(x, n, 0.f, s), "fill");
        XS(hipMemcpyAsync(r, b, n * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
        XS(xrl::dots(n, b, b, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_BB, s), "dots");
        XS(read_slots(), "sync");
        bn = sqrt(host[S_BB]);
        if (bn == 0.0) {
            info->converged = 1;
            goto done;
        }
        while (true) {
            if (rel <= tol) {
                // confirm with the explicitly computed residual r = b - M x
                XM(M(x, q));
                XS(xrl::axpy2(n, slots, S_BB, S_BB, -1, b, q, r, nullptr, nullptr, nullptr, s), "axpy");
                XS(xrl::dots(n, r, r, nullptr, nullptr, nullptr, nullptr, dpart, slots, T_RRN, s), "dots");
                XS(read_slots(), "sync");
                rel = sqrt(host[T_RRN]) / bn;
                if (rel <= tol) {
                    confirmed = true;
                    break;
                }
                fresh = true;   // restart from the true residual
            }
            if (info->iterations >= maxit) break;
            if (fresh) {
                // p = z = P r, <r, z>
                XM(P(r, z));
                XS(xrl::dots(n, r, z, nullptr, nullptr, nullptr, nullptr, dpart, slots, T_RZ, s), "dots");
                XS(hipMemcpyAsync(p, z, n * sizeof(float), hipMemcpyDeviceToDevice, s), "hipMemcpyAsync");
                fresh = false;
            }
            XM(M(p, q));
            XS(xrl::dots(n, p, q, nullptr, nullptr, nullptr, nullptr, dpart, slots, S_PQ, s), "dots");
            // alpha = <r, z> / <p, M p>; x += alpha p; r -= alpha M p
            XS(xrl::axpy2(n, slots, T_RZ, S_PQ, 1, x, p, x, r, q, r, s), "axpy");
            XM(P(r, z));
            // <r, z> (new) and <r, r>
            XS(xrl::dots(n, r, z, r, r, nullptr, nullptr, dpart, slots, T_RZN, s), "dots");
            // p = z + (<r, z>_new / <r, z>) p
            XS(xrl::direction(n, slots, T_RZN, -1, T_RZ, z, p, p, s), "direction");
            XS(xrl::copy_slot(slots, T_RZ, T_RZN, s), "copy");
            XS(read_slots(), "sync");
            rel = sqrt(host[T_RRN]) / bn;
            info->iterations += 1;
            if (history && hist_n < history_cap) history[hist_n++] = rel;
        }
        if (!confirmed) {
            XM(M(x, q));
            XS(xrl::axpy2(n, slots, S_BB, S_BB, -1, b, q, r, nullptr, nullptr, nullptr, s), "axpy");
            XS(xrl::dots(n, r, r, nullptr, nullptr, nullptr, nullptr, dpart, slots, T_RRN, s), "dots");
            XS(read_slots(), "sync");
            rel = sqrt(host[T_RRN]) / bn;
        }
        info->rel_residual = rel;
        info->converged = rel <= tol ? 1 : 0;
    }
done:
    (void)hipStreamSynchronize(s);
    return st;
}

}  // extern "C"
