// xrt_learn_internal.h -- kernels behind the learned preconditioner (a small
// U-Net on bf16 matrix cores) and the regularised normal-equations solver.
// Shared by xrt_learn.hip (kernels, launchers) and xrt_learn.cpp (network and
// solver orchestration).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace xrl {

// Feature maps are NHWC bfloat16 (raw 16-bit patterns in memory).  A view is a
// pointer to channel 0 of the first pixel plus the element distance between
// consecutive pixels (>= the number of channels; a concatenation buffer holds
// two views with one pitch).  Pointers and pitches are multiples of 8 elements.
struct View {
    uint16_t* p;
    int pitch;
};
struct CView {
    const uint16_t* p;
    int pitch;
};

// 3x3 convolution, zero padding, no bias:
//   y[b,h,w,o] = act( sum_{tap,i} x[b, h+ky-1, w+kx-1, i] * w[tap][o][i] ),
// tap = 3 ky + kx.  act: optional ReLU, then optional mask (y = 0 where the
// mask tensor is <= 0; the mask has the output's shape and its own pitch).
// The input x is read in one of three ways (in_mode), so that a pooling or an
// upsampling feeding the convolution need not be written out first:
//   kConvPlain  x[b, h, w, i] at the output's size;
//   kConvPool   the 2x2 average of x at twice the output's size, rounded to
//               bf16 exactly as avgpool2 writes it;
//   kConvUpcat  channels i < cin/2 from x at the output's size, channels
//               i >= cin/2 from x2 at half the size (nearest neighbour),
//               i.e. the concatenation [x, upsample2(x2)] that upsample2
//               builds.
enum { kConvPlain = 0, kConvPool = 1, kConvUpcat = 2 };
struct ConvArgs {
    CView x;
    const uint16_t* w = nullptr;   // [9][cout][cin]
    void* y = nullptr;             // bf16 view or float [pixels][ypitch]
    int ypitch = 0;
    CView mask{nullptr, 0};        // p == nullptr: none
    int B = 0, H = 0, W = 0, cin = 0, cout = 0;
    int relu = 0;
    int in_mode = kConvPlain;
    CView x2{nullptr, 0};          // kConvUpcat: the half-size input
    // split of the input-channel reduction over workgroups (set by conv3x3):
    // ksplit > 1 writes fp32 partial sums kpart[k][pixel][cout], then a
    // reduction applies the activation and mask
    int ksplit = 1;
    float* kpart = nullptr;
};

// Weight gradient of the convolution above: per region of pixels, partial
// sums part[region][9][cout][cin] of g[b,h,w,o] * x[b,h+ky-1,w+kx-1,i].
struct WgradArgs {
    CView x, g;
    float* part;
    int B, H, W, cin, cout;
    int rows;            // image rows per region (even)
};

// `ws` (may be null: no split) is a workspace of ws_floats floats for the
// split-K partial sums
hipError_t conv3x3(const ConvArgs& a, bool f32_out, float* ws, int64_t ws_floats, hipStream_t s);
// the largest workspace conv3x3 can use for this shape (0: it never splits)
int64_t conv3x3_ws_floats(int B, int H, int W, int cin, int cout);
hipError_t conv3x3_wgrad(const WgradArgs& a, int* n_regions, hipStream_t s);
int wgrad_rows(int B, int H, int W, int cin, int cout);
int64_t wgrad_regions(int B, int H, int W, int rows);
// pixels per region of the first and last layers' weight gradients
int per_block_pixels(int64_t npix);

// first layer (one input channel, fp32, scaled per image) and its weight gradient
hipError_t conv_in(const float* x, const float* scale, const uint16_t* w /*[9][c]*/, View y, int c,
                   int B, int H, int W, bool relu, hipStream_t s);
hipError_t conv_in_wgrad(const float* x, const float* scale, CView g, int c, int B, int H, int W,
                         float* part, int* n_regions, hipStream_t s);
// 1x1 output layer c -> 1 (fp32 out), its input gradient (masked by d > 0 if mask) and weight gradient
// y[p] = sum_i d[p, i] w[i]; with scale != nullptr the output is unscaled on the
// way out, y[p] = sum * (gain / scale[p / img_npix]), as unscale does.
hipError_t conv_out(CView d, const uint16_t* w, int c, float* y, int npix, hipStream_t s,
                    const float* scale = nullptr, float gain = 1.f, int64_t img_npix = 1);
hipError_t conv_out_bwd(CView d, const uint16_t* w, const float* gy, int c, View gd, int npix, bool mask,
                        hipStream_t s);
hipError_t conv_out_wgrad(CView d, const float* gy, int c, int npix, float* part, int* n_regions,
                          hipStream_t s);

// 2x2 average pool; its transpose added into g (masked by e > 0 unless e.p is null); nearest 2x
// upsampling; its transpose (2x2 sum).  H, W are the FINE sizes.
hipError_t avgpool2(CView x, View y, int c, int B, int H, int W, hipStream_t s);
hipError_t avgpool2_T_add(CView gc, View g, CView e, int c, int B, int H, int W, hipStream_t s);
hipError_t upsample2(CView x, View y, int c, int B, int H, int W, hipStream_t s);
hipError_t upsample2_T(CView g, View y, int c, int B, int H, int W, hipStream_t s);

// out[e] = sum_r part[r * n + e]
hipError_t reduce_parts(const float* part, int nreg, int64_t n, float* out, hipStream_t s);

// per image: scale[b] = 1/rms(r_b); if e: tn[b] = (scale[b]/gain)^2 * sum e_b^2
// part: image_parts() * 2 * B doubles of workspace
int image_parts();
hipError_t image_stats(const float* r, const float* e, int B, int64_t npix, float gain, float* scale,
                       float* tn, double* part, hipStream_t s);
// loss = mean_b ||y_b - (scale_b/gain) e_b||^2 / tn_b; gy = its gradient; loss to *loss (device)
hipError_t loss_grad(const float* y, const float* e, const float* scale, const float* tn, int B,
                     int64_t npix, float gain, float* gy, float* part, float* loss, hipStream_t s);
// residual-space loss: d = q - r, rr[b] = ||r_b||^2, lb[b] = ||d_b||^2 / rr[b], *loss = mean_b lb[b]
hipError_t resid_stats(const float* q, const float* r, float* d, int B, int64_t npix, float* rr, float* lb,
                       float* loss, double* part, hipStream_t s);
// energy-norm loss: d = q - r, er[b] = e_b^T r_b (= e_b^T M e_b), lb[b] =
// (z_b - e_b)^T M (z_b - e_b) / er[b] from q = M z, *loss = mean_b lb[b];
// part: 3 * image_parts() * B doubles.  Its gradient w.r.t. the network
// output is resid_grad(d, scale, er, ...) (M symmetric: 2 (M z - r) / er).
hipError_t energy_stats(const float* z, const float* q, const float* r, const float* e, float* d, int B,
                        int64_t npix, float* er, float* lb, float* loss, double* part, hipStream_t s);
// its gradient w.r.t. the normalised network output: gy = md * 2 gain / (scale[b] B rr[b])
hipError_t resid_grad(const float* md, const float* scale, const float* rr, int B, int64_t npix, float gain,
                      float* gy, hipStream_t s);
// z = y * gain / scale[b]
hipError_t unscale(const float* y, const float* scale, int B, int64_t npix, float gain, float* z,
                   hipStream_t s);

// Adam on the fp32 master parameters; then the bf16 copies of a layer
hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                float eps, float c1, float c2, hipStream_t s);
// wf[tap][o][i] = bf16(p[tap][o][i]); if wb: wb[8-tap][i][o] = wf[tap][o][i]
hipError_t pack_weights(const float* p, int taps, int cout, int cin, uint16_t* wf, uint16_t* wb,
                        hipStream_t s);
hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s);
// out[v][j] = sum_k f[k] in[v][j + k - K/2] over each view's nbins samples (zero outside)
hipError_t sino_filter(const float* in, int64_t nviews, int nbins, const float* f, int K, float* out, hipStream_t s);
// z += mu r
hipError_t add_scaled(int64_t n, float mu, const float* r, float* z, hipStream_t s);
// wb[taps-1-tap][i][o] = w[tap][o][i]
hipError_t flip_weights(const uint16_t* w, int taps, int cout, int cin, uint16_t* wb, hipStream_t s);

// ---- solver vector kernels (fp32 vectors, fp64 scalars on the device)
// out (+)= lam * L^T L c on an [ny][nx] grid (forward differences, Neumann)
hipError_t reg_apply(const float* c, float* out, int nx, int ny, float lam, bool accumulate,
                     hipStream_t s);
// slot[k] = <a_k, b_k> for the non-null pairs (k < 3); fp64 partials then one final pass
hipError_t dots(int64_t n, const float* a0, const float* b0, const float* a1, const float* b1,
                const float* a2, const float* b2, double* part, double* slots, int slot0,
                hipStream_t s);
// y = x + (num/den) * d ; if y2: y2 = x2 - (num/den) * d2   (scalars read from `slots`)
hipError_t axpy2(int64_t n, const double* slots, int num, int den, int sign_num,
                 const float* x, const float* d, float* y,
                 const float* x2, const float* d2, float* y2, hipStream_t s);
// out = z + beta p, beta = (slots[a] - slots[b]) / slots[c] (b < 0: no subtraction;
// c < 0: out = z and p is not read).  out may alias p.
hipError_t direction(int64_t n, const double* slots, int a, int b, int c, const float* z, const float* p,
                     float* out, hipStream_t s);
// a list of device vectors passed by value to a kernel
constexpr int kMaxVecs = 16;
struct VecList {
    const float* v[kMaxVecs];
};
// slots[slot0 + j] = <x, ys_j>, j < k <= kMaxVecs
hipError_t dots_multi(int64_t n, const float* x, const VecList& ys, int k, double* part, double* slots, int slot0,
                      hipStream_t s);
// out = z - sum_{j<k} (slots[a + j] / slots[b + j]) ps_j   (out may alias z)
hipError_t orth(int64_t n, const double* slots, int a, int b, int k, const float* z, const VecList& ps, float* out,
                hipStream_t s);
// slots[dst] = slots[src]
hipError_t copy_slot(double* slots, int dst, int src, hipStream_t s);
int dots_parts();

}  // namespace xrl
