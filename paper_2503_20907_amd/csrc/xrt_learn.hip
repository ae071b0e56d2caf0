// xrt_learn.hip -- gfx950 kernels of the learned preconditioner and of the
// regularised normal-equations solver.
//
// The network's 3x3 convolutions run on the bf16 matrix cores
// (v_mfma_f32_32x32x16_bf16, fp32 accumulation) as implicit GEMMs:
//   forward / input gradient:  D[o][pixel] = sum_{tap, i} W[tap][o][i] X[pixel + tap][i]
//   weight gradient:           D[o][i]     = sum_{pixel}  G[pixel][o] X[pixel + tap][i]
// Operand layout of the 32x32x16 instruction (lane l, 8 bf16 per lane):
// A row l%32, k = 8 (l/32) .. +7; B column l%32, same k; result register i
// of lane l holds row 8 (i/4) + 4 (l/32) + i%4, column l%32.
// Everything else (first and last layer, pooling, loss, Adam, CG vector
// updates) is memory-bound and written as plain coalesced VALU kernels.
#include "xrt_learn_internal.h"

namespace xrl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ float bf2f(uint32_t h) { return __uint_as_float(h << 16); }
__device__ __forceinline__ uint32_t f2bf(float f)
{
    // round to nearest, ties to even (finite inputs)
    const uint32_t u = __float_as_uint(f);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ float lo_bf(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float hi_bf(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ __forceinline__ uint32_t pack2(float a, float b) { return f2bf(a) | (f2bf(b) << 16); }
__device__ __forceinline__ bool bf_pos(uint32_t h16) { return (h16 & 0x8000u) == 0 && (h16 & 0x7FFFu) != 0; }

__device__ __forceinline__ u32x4 ld16(const uint16_t* p) { return *reinterpret_cast<const u32x4*>(p); }
__device__ __forceinline__ void st16(uint16_t* p, u32x4 v) { *reinterpret_cast<u32x4*>(p) = v; }
__device__ __forceinline__ bf16x8 frag(const uint16_t* p) { return __builtin_bit_cast(bf16x8, ld16(p)); }

// ------------------------------------------------------------- 3x3 convolution
constexpr int kTW = 64;         // output pixels per tile row
constexpr int kTR = 4;          // output rows per tile (one per wave)
constexpr int kXW = kTW + 2;    // staged input pixels per row (1-pixel halo)

// 64-byte LDS rows of 32 channels; the 16-byte slot q is XOR-swizzled with the
// row so that 8 consecutive rows read at the same q hit 8 distinct bank groups.
__device__ __forceinline__ int swz(int row, int q) { return row * 32 + 8 * (q ^ ((row >> 1) & 3)); }

// 8 input channels from ch of the convolution's input at (b, gh, gw), read as
// ConvArgs::in_mode says
template <int MODE>
__device__ __forceinline__ u32x4 conv_in8(const ConvArgs& a, int b, int gh, int gw, int ch)
{
    if constexpr (MODE == kConvPool) {
        const int H2 = 2 * a.H, W2 = 2 * a.W;
        float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const size_t pf = (size_t)(b * H2 + 2 * gh + (t >> 1)) * W2 + 2 * gw + (t & 1);
            const u32x4 v = ld16(a.x.p + pf * a.x.pitch + ch);
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += lo_bf(v[k]);
                s[2 * k + 1] += hi_bf(v[k]);
            }
        }
        return u32x4{pack2(0.25f * s[0], 0.25f * s[1]), pack2(0.25f * s[2], 0.25f * s[3]),
                     pack2(0.25f * s[4], 0.25f * s[5]), pack2(0.25f * s[6], 0.25f * s[7])};
    } else if constexpr (MODE == kConvUpcat) {
        const int half = a.cin / 2;
        if (ch >= half) {
            const size_t pc = (size_t)(b * (a.H / 2) + gh / 2) * (a.W / 2) + gw / 2;
            return ld16(a.x2.p + pc * a.x2.pitch + ch - half);
        }
    }
    return ld16(a.x.p + ((size_t)(b * a.H + gh) * a.W + gw) * a.x.pitch + ch);
}

template <int COT, bool F32OUT, int MODE>
__global__ __launch_bounds__(256) void k_conv3x3(ConvArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t xs[(kTR + 2) * kXW * 32];
    __shared__ __attribute__((aligned(16))) uint16_t ws[9 * COT * 32];
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, n = l & 31, kg = l >> 5;
    const int ntw = (a.W + kTW - 1) / kTW;
    const int w0 = (blockIdx.x % ntw) * kTW, h0 = (blockIdx.x / ntw) * kTR;
    const int ncb = a.cout / COT;
    const int b = blockIdx.y, co0 = (blockIdx.z % ncb) * COT, kp = blockIdx.z / ncb;
    const int nch = a.cin / 32;
    const int c_lo = (int)((int64_t)kp * nch / a.ksplit), c_hi = (int)((int64_t)(kp + 1) * nch / a.ksplit);
    f32x16 acc[COT / 32][2];
#pragma unroll
    for (int i = 0; i < COT / 32; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            for (int k = 0; k < 16; ++k) acc[i][j][k] = 0.f;

    for (int ci0 = 32 * c_lo; ci0 < 32 * c_hi; ci0 += 32) {
        __syncthreads();
        for (int v = tid; v < (kTR + 2) * kXW * 4; v += 256) {
            const int q = v & 3, pix = v >> 2;
            const int r = pix / kXW, c = pix - r * kXW;
            const int gh = h0 + r - 1, gw = w0 + c - 1;
            u32x4 val = {0u, 0u, 0u, 0u};
            if (gh >= 0 && gh < a.H && gw >= 0 && gw < a.W) val = conv_in8<MODE>(a, b, gh, gw, ci0 + 8 * q);
            st16(xs + swz(pix, q), val);
        }
        for (int v = tid; v < 9 * COT * 4; v += 256) {
            const int q = v & 3, row = v >> 2;
            const int tap = row / COT, co = row - tap * COT;
            st16(ws + swz(row, q), ld16(a.w + ((size_t)tap * a.cout + co0 + co) * a.cin + ci0 + 8 * q));
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int ky = tap / 3, kx = tap % 3;
#pragma unroll
            for (int ks = 0; ks < 2; ++ks) {
                const int q = 2 * ks + kg;
                bf16x8 bx[2], aw[COT / 32];
#pragma unroll
                for (int pb = 0; pb < 2; ++pb)
                    bx[pb] = frag(xs + swz((wv + ky) * kXW + pb * 32 + n + kx, q));
#pragma unroll
                for (int cb = 0; cb < COT / 32; ++cb)
                    aw[cb] = frag(ws + swz(tap * COT + cb * 32 + n, q));
#pragma unroll
                for (int cb = 0; cb < COT / 32; ++cb)
#pragma unroll
                    for (int pb = 0; pb < 2; ++pb)
                        acc[cb][pb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(aw[cb], bx[pb], acc[cb][pb], 0, 0, 0);
            }
        }
    }

    const int h = h0 + wv;
    if (h >= a.H) return;
#pragma unroll
    for (int pb = 0; pb < 2; ++pb) {
        const int px = w0 + pb * 32 + n;
        if (px >= a.W) continue;
        const size_t pix = (size_t)(b * a.H + h) * a.W + px;
        if (a.ksplit > 1) {
            // raw partial sums; the reduction applies the epilogue
            float* kq = a.kpart + ((size_t)kp * a.B * a.H * a.W + pix) * a.cout;
#pragma unroll
            for (int cb = 0; cb < COT / 32; ++cb)
#pragma unroll
                for (int g = 0; g < 4; ++g) {
                    const int co = co0 + cb * 32 + 8 * g + 4 * kg;
                    *reinterpret_cast<float4*>(kq + co) = make_float4(acc[cb][pb][4 * g], acc[cb][pb][4 * g + 1],
                                                                      acc[cb][pb][4 * g + 2], acc[cb][pb][4 * g + 3]);
                }
            continue;
        }
#pragma unroll
        for (int cb = 0; cb < COT / 32; ++cb) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                const int co = co0 + cb * 32 + 8 * g + 4 * kg;
                float v[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    v[j] = acc[cb][pb][4 * g + j];
                    if (a.relu) v[j] = fmaxf(v[j], 0.f);
                }
                if (a.mask.p) {
                    const u32x2 m = *reinterpret_cast<const u32x2*>(a.mask.p + pix * a.mask.pitch + co);
                    if (!bf_pos(m[0] & 0xFFFFu)) v[0] = 0.f;
                    if (!bf_pos(m[0] >> 16)) v[1] = 0.f;
                    if (!bf_pos(m[1] & 0xFFFFu)) v[2] = 0.f;
                    if (!bf_pos(m[1] >> 16)) v[3] = 0.f;
                }
                if constexpr (F32OUT) {
                    float* y = static_cast<float*>(a.y) + pix * a.ypitch + co;
                    *reinterpret_cast<float4*>(y) = make_float4(v[0], v[1], v[2], v[3]);
                } else {
                    uint16_t* y = static_cast<uint16_t*>(a.y) + pix * a.ypitch + co;
                    *reinterpret_cast<u32x2*>(y) = u32x2{pack2(v[0], v[1]), pack2(v[2], v[3])};
                }
            }
        }
    }
}

// Sum of the split-K partials, then the convolution's epilogue (ReLU, mask,
// store).  Thread per (pixel, 4 output channels).
__global__ void k_conv_reduce(ConvArgs a, int f32out)
{
    const int64_t npix = (int64_t)a.B * a.H * a.W;
    const int nq = a.cout / 4;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npix * nq) return;
    const int co = 4 * (int)(idx % nq);
    const int64_t pix = idx / nq;
    float4 v = *reinterpret_cast<const float4*>(a.kpart + pix * a.cout + co);
    for (int k = 1; k < a.ksplit; ++k) {
        const float4 u = *reinterpret_cast<const float4*>(a.kpart + ((int64_t)k * npix + pix) * a.cout + co);
        v.x += u.x;
        v.y += u.y;
        v.z += u.z;
        v.w += u.w;
    }
    float w4[4] = {v.x, v.y, v.z, v.w};
    if (a.relu)
        for (int j = 0; j < 4; ++j) w4[j] = fmaxf(w4[j], 0.f);
    if (a.mask.p) {
        const u32x2 m = *reinterpret_cast<const u32x2*>(a.mask.p + pix * a.mask.pitch + co);
        if (!bf_pos(m[0] & 0xFFFFu)) w4[0] = 0.f;
        if (!bf_pos(m[0] >> 16)) w4[1] = 0.f;
        if (!bf_pos(m[1] & 0xFFFFu)) w4[2] = 0.f;
        if (!bf_pos(m[1] >> 16)) w4[3] = 0.f;
    }
    if (f32out) {
        *reinterpret_cast<float4*>(static_cast<float*>(a.y) + pix * a.ypitch + co) = make_float4(w4[0], w4[1], w4[2], w4[3]);
    } else {
        *reinterpret_cast<u32x2*>(static_cast<uint16_t*>(a.y) + pix * a.ypitch + co) =
            u32x2{pack2(w4[0], w4[1]), pack2(w4[2], w4[3])};
    }
}

// ------------------------------------------------------------ weight gradient
constexpr int kGP = 136;   // LDS pitch of a gradient row: 2 image rows x 64 pixels + 8
constexpr int kXR = 72;    // LDS pitch of an input row: 64 pixels + 8

// v[t] holds 8 channels of pixel t; o[c] receives 8 pixels of channel c.
__device__ __forceinline__ void transpose8(const u32x4 (&v)[8], u32x4 (&o)[8])
{
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t A = v[2 * e][d], B = v[2 * e + 1][d];
            o[2 * d][e] = (A & 0xFFFFu) | (B << 16);
            o[2 * d + 1][e] = (A >> 16) | (B & 0xFFFF0000u);
        }
}

// One workgroup: a region of `rows` image rows x 64 columns of one image, a
// 32 x 32 (output channel, input channel) block, all 9 taps.  Pixels are the
// reduction dimension, so both operands are staged transposed (pixels
// contiguous) in LDS; the input is staged three times, shifted by kx - 1
// columns, so every fragment read is 16-byte aligned.
__global__ __launch_bounds__(256) void k_wgrad(WgradArgs a)
{
    __shared__ __attribute__((aligned(16))) uint16_t gT[32 * kGP];          // [o][row*64 + px]
    __shared__ __attribute__((aligned(16))) uint16_t xT[3 * 4 * 32 * kXR];  // [kx][row][i][px]
    const int tid = threadIdx.x, wv = tid >> 6, l = tid & 63, n = l & 31, kg = l >> 5;
    const int ntw = (a.W + 63) / 64, nrg = (a.H + a.rows - 1) / a.rows;
    const int reg = blockIdx.x;
    const int wt = reg % ntw, rg = (reg / ntw) % nrg, b = reg / (ntw * nrg);
    const int w0 = wt * 64;
    const int nci = a.cin / 32;
    const int co0 = (blockIdx.y / nci) * 32, ci0 = (blockIdx.y % nci) * 32;
    f32x16 acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t)
        for (int k = 0; k < 16; ++k) acc[t][k] = 0.f;

    const int hend = min(a.H, (rg + 1) * a.rows);
    for (int h = rg * a.rows; h < hend; h += 2) {
        __syncthreads();
        for (int it = tid; it < 64 + 384; it += 256) {
            u32x4 v[8];
            uint16_t* dst;
            int stride;
            if (it < 64) {
                const int r = it >> 5, j8 = (it >> 2) & 7, q = it & 3;
                const int gh = h + r;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int px = w0 + 8 * j8 + t;
                    v[t] = u32x4{0u, 0u, 0u, 0u};
                    if (gh < a.H && px < a.W)
                        v[t] = ld16(a.g.p + ((size_t)(b * a.H + gh) * a.W + px) * a.g.pitch + co0 + 8 * q);
                }
                dst = gT + (8 * q) * kGP + r * 64 + 8 * j8;
                stride = kGP;
            } else {
                const int k = it - 64, dx = k >> 7, r = (k >> 5) & 3, j8 = (k >> 2) & 7, q = k & 3;
                const int gh = h + r - 1;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int px = w0 + 8 * j8 + t + dx - 1;
                    v[t] = u32x4{0u, 0u, 0u, 0u};
                    if (gh >= 0 && gh < a.H && px >= 0 && px < a.W)
                        v[t] = ld16(a.x.p + ((size_t)(b * a.H + gh) * a.W + px) * a.x.pitch + ci0 + 8 * q);
                }
                dst = xT + ((dx * 4 + r) * 32 + 8 * q) * kXR + 8 * j8;
                stride = kXR;
            }
            u32x4 o[8];
            transpose8(v, o);
#pragma unroll
            for (int c = 0; c < 8; ++c) st16(dst + c * stride, o[c]);
        }
        __syncthreads();
        const int r = wv >> 1;
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const int k0 = (wv & 1) * 32 + ks * 16 + 8 * kg;
            const bf16x8 A = frag(gT + n * kGP + r * 64 + k0);
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int ky = tap / 3, kx = tap % 3;
                const bf16x8 B = frag(xT + ((kx * 4 + r + ky) * 32 + n) * kXR + k0);
                acc[tap] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, acc[tap], 0, 0, 0);
            }
        }
    }

    // sum the four waves' accumulators in LDS (one wave at a time)
    __syncthreads();
    float* red = reinterpret_cast<float*>(xT);   // [9][32][32]
    for (int w = 0; w < 4; ++w) {
        if (wv == w) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int m = 8 * (i >> 2) + 4 * kg + (i & 3);
                    const int idx = (tap * 32 + m) * 32 + n;
                    red[idx] = (w ? red[idx] : 0.f) + acc[tap][i];
                }
        }
        __syncthreads();
    }
    float* out = a.part + (size_t)reg * 9 * a.cout * a.cin;
    for (int e = tid; e < 9 * 1024; e += 256) {
        const int tap = e >> 10, m = (e >> 5) & 31, nn = e & 31;
        out[((size_t)tap * a.cout + co0 + m) * a.cin + ci0 + nn] = red[e];
    }
}

// ------------------------------------------------------ first and last layer
__global__ __launch_bounds__(256) void k_conv_in(const float* x, const float* scale, const uint16_t* w, View y,
                                                 int c, int B, int H, int W, int relu)
{
    __shared__ float wl[9 * 256];
    for (int i = threadIdx.x; i < 9 * c; i += 256) wl[i] = bf2f(w[i]);
    __syncthreads();
    const int ng = c / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * H * W * ng) return;
    const int g = (int)(idx % ng);
    const int64_t pix = idx / ng;
    const int px = (int)(pix % W), h = (int)((pix / W) % H), b = (int)(pix / ((int64_t)W * H));
    const float s = scale[b];
    float xin[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) {
        const int hh = h + t / 3 - 1, ww = px + t % 3 - 1;
        xin[t] = (hh >= 0 && hh < H && ww >= 0 && ww < W) ? x[((int64_t)b * H + hh) * W + ww] * s : 0.f;
    }
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        float acc = 0.f;
#pragma unroll
        for (int t = 0; t < 9; ++t) acc = fmaf(xin[t], wl[t * c + 8 * g + j], acc);
        v[j] = relu ? fmaxf(acc, 0.f) : acc;
    }
    st16(y.p + pix * y.pitch + 8 * g,
         u32x4{pack2(v[0], v[1]), pack2(v[2], v[3]), pack2(v[4], v[5]), pack2(v[6], v[7])});
}

// part[block][9][c]; thread: channel tid % c, pixel slot tid / c
__global__ __launch_bounds__(256) void k_conv_in_wgrad(const float* x, const float* scale, CView g, int c,
                                                       int B, int H, int W, int per_block, float* part)
{
    __shared__ float red[256 * 9];
    const int co = threadIdx.x % c, slot = threadIdx.x / c, nslot = 256 / c;
    const int64_t npix = (int64_t)B * H * W;
    const int64_t p0 = (int64_t)blockIdx.x * per_block, p1 = min(npix, p0 + per_block);
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // the pixel's coordinates, divided out once and then advanced by nslot
    int px = 0, h = 0, b = 0;
    if (p0 + slot < p1) {
        const int64_t q = p0 + slot;
        px = (int)(q % W);
        h = (int)((q / W) % H);
        b = (int)(q / ((int64_t)W * H));
    }
    for (int64_t p = p0 + slot; p < p1; p += nslot) {
        const int cx = px, ch = h, cb = b;
        px += nslot;
        while (px >= W) {
            px -= W;
            if (++h == H) {
                h = 0;
                ++b;
            }
        }
        // no branch on gv == 0: the x loads then need not wait for g's
        const float gs = bf2f(g.p[p * g.pitch + co]) * scale[cb];
#pragma unroll
        for (int t = 0; t < 9; ++t) {
            const int hh = ch + t / 3 - 1, ww = cx + t % 3 - 1;
            if (hh >= 0 && hh < H && ww >= 0 && ww < W) acc[t] = fmaf(gs, x[((int64_t)cb * H + hh) * W + ww], acc[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < 9; ++t) red[(slot * 9 + t) * c + co] = acc[t];
    __syncthreads();
    for (int e = threadIdx.x; e < 9 * c; e += 256) {
        float s = 0.f;
        for (int k = 0; k < nslot; ++k) s += red[k * 9 * c + e];
        part[(int64_t)blockIdx.x * 9 * c + e] = s;
    }
}

__global__ void k_conv_out(CView d, const uint16_t* w, int c, float* y, int64_t npix, const float* scale, float gain,
                           int64_t img_npix)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    float acc = 0.f;
    for (int g = 0; g < c / 8; ++g) {
        const u32x4 v = ld16(d.p + p * d.pitch + 8 * g);
        const u32x4 ww = ld16(w + 8 * g);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            acc = fmaf(lo_bf(v[k]), lo_bf(ww[k]), acc);
            acc = fmaf(hi_bf(v[k]), hi_bf(ww[k]), acc);
        }
    }
    y[p] = scale ? acc * (gain / scale[p / img_npix]) : acc;
}

__global__ void k_conv_out_bwd(CView d, const uint16_t* w, const float* gy, int c, View gd, int64_t npix, int mask)
{
    const int ng = c / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= npix * ng) return;
    const int g = (int)(idx % ng);
    const int64_t p = idx / ng;
    const float gv = gy[p];
    const u32x4 v = ld16(d.p + p * d.pitch + 8 * g);
    const u32x4 ww = ld16(w + 8 * g);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float a0 = (!mask || bf_pos(v[k] & 0xFFFFu)) ? lo_bf(ww[k]) * gv : 0.f;
        const float a1 = (!mask || bf_pos(v[k] >> 16)) ? hi_bf(ww[k]) * gv : 0.f;
        o[k] = pack2(a0, a1);
    }
    st16(gd.p + p * gd.pitch + 8 * g, o);
}

__global__ __launch_bounds__(256) void k_conv_out_wgrad(CView d, const float* gy, int c, int64_t npix,
                                                        int per_block, float* part)
{
    __shared__ float red[256];
    const int co = threadIdx.x % c, slot = threadIdx.x / c, nslot = 256 / c;
    const int64_t p0 = (int64_t)blockIdx.x * per_block, p1 = min(npix, p0 + per_block);
    float acc = 0.f;
    for (int64_t p = p0 + slot; p < p1; p += nslot) acc = fmaf(bf2f(d.p[p * d.pitch + co]), gy[p], acc);
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < c) {
        float s = 0.f;
        for (int k = 0; k < nslot; ++k) s += red[k * c + threadIdx.x];
        part[(int64_t)blockIdx.x * c + threadIdx.x] = s;
    }
}

// ------------------------------------------------------- pooling / upsampling
// thread per (coarse pixel, 8 channels); H, W fine sizes
__global__ void k_avgpool2(CView x, View y, int c, int B, int H, int W)
{
    const int ng = c / 8, Hc = H / 2, Wc = W / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * Hc * Wc * ng) return;
    const int g = (int)(idx % ng);
    const int64_t pc = idx / ng;
    const int xc = (int)(pc % Wc), hc = (int)((pc / Wc) % Hc), b = (int)(pc / ((int64_t)Wc * Hc));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t pf = ((int64_t)b * H + 2 * hc + (t >> 1)) * W + 2 * xc + (t & 1);
        const u32x4 v = ld16(x.p + pf * x.pitch + 8 * g);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[2 * k] += lo_bf(v[k]);
            s[2 * k + 1] += hi_bf(v[k]);
        }
    }
    st16(y.p + pc * y.pitch + 8 * g, u32x4{pack2(0.25f * s[0], 0.25f * s[1]), pack2(0.25f * s[2], 0.25f * s[3]),
                                           pack2(0.25f * s[4], 0.25f * s[5]), pack2(0.25f * s[6], 0.25f * s[7])});
}

// thread per (fine pixel, 8 channels): g += [e > 0] * gc(coarse) / 4
__global__ void k_avgpool2_T_add(CView gc, View g, CView e, int c, int B, int H, int W)
{
    const int ng = c / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * H * W * ng) return;
    const int gi = (int)(idx % ng);
    const int64_t pf = idx / ng;
    const int xf = (int)(pf % W), hf = (int)((pf / W) % H), b = (int)(pf / ((int64_t)W * H));
    const int64_t pc = ((int64_t)b * (H / 2) + hf / 2) * (W / 2) + xf / 2;
    const u32x4 vc = ld16(gc.p + pc * gc.pitch + 8 * gi);
    const u32x4 ve = e.p ? ld16(e.p + pf * e.pitch + 8 * gi) : u32x4{0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};
    uint16_t* gp = g.p + pf * g.pitch + 8 * gi;
    const u32x4 vg = ld16(gp);
    u32x4 o;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const float a0 = lo_bf(vg[k]) + (bf_pos(ve[k] & 0xFFFFu) ? 0.25f * lo_bf(vc[k]) : 0.f);
        const float a1 = hi_bf(vg[k]) + (bf_pos(ve[k] >> 16) ? 0.25f * hi_bf(vc[k]) : 0.f);
        o[k] = pack2(a0, a1);
    }
    st16(gp, o);
}

// thread per (fine pixel, 8 channels)
__global__ void k_upsample2(CView x, View y, int c, int B, int H, int W)
{
    const int ng = c / 8;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * H * W * ng) return;
    const int g = (int)(idx % ng);
    const int64_t pf = idx / ng;
    const int xf = (int)(pf % W), hf = (int)((pf / W) % H), b = (int)(pf / ((int64_t)W * H));
    const int64_t pc = ((int64_t)b * (H / 2) + hf / 2) * (W / 2) + xf / 2;
    st16(y.p + pf * y.pitch + 8 * g, ld16(x.p + pc * x.pitch + 8 * g));
}

// thread per (coarse pixel, 8 channels): y = sum of the 4 fine values
__global__ void k_upsample2_T(CView gf, View y, int c, int B, int H, int W)
{
    const int ng = c / 8, Hc = H / 2, Wc = W / 2;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)B * Hc * Wc * ng) return;
    const int g = (int)(idx % ng);
    const int64_t pc = idx / ng;
    const int xc = (int)(pc % Wc), hc = (int)((pc / Wc) % Hc), b = (int)(pc / ((int64_t)Wc * Hc));
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int64_t pf = ((int64_t)b * H + 2 * hc + (t >> 1)) * W + 2 * xc + (t & 1);
        const u32x4 v = ld16(gf.p + pf * gf.pitch + 8 * g);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            s[2 * k] += lo_bf(v[k]);
            s[2 * k + 1] += hi_bf(v[k]);
        }
    }
    st16(y.p + pc * y.pitch + 8 * g,
         u32x4{pack2(s[0], s[1]), pack2(s[2], s[3]), pack2(s[4], s[5]), pack2(s[6], s[7])});
}

// ------------------------------------------------------------ reductions etc.
// out[e] = sum over regions r of part[r][e], in a fixed order: a workgroup
// takes 32 consecutive e; its 8 thread groups each sum a contiguous eighth of
// the regions (four interleaved running sums, combined pairwise), and the
// eight group sums are added in group order.  The result does not depend on
// the schedule.
constexpr int kRedE = 32, kRedG = 8;
__global__ __launch_bounds__(256) void k_reduce_parts(const float* part, int nreg, int64_t n, float* out)
{
    __shared__ float sh[kRedG][kRedE];
    const int j = threadIdx.x % kRedE, grp = threadIdx.x / kRedE;
    const int64_t e = (int64_t)blockIdx.x * kRedE + j;
    const int r0 = (int)((int64_t)grp * nreg / kRedG), r1 = (int)((int64_t)(grp + 1) * nreg / kRedG);
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    if (e < n) {
        int r = r0;
        for (; r + 4 <= r1; r += 4) {
            a0 += part[(int64_t)r * n + e];
            a1 += part[(int64_t)(r + 1) * n + e];
            a2 += part[(int64_t)(r + 2) * n + e];
            a3 += part[(int64_t)(r + 3) * n + e];
        }
        for (; r < r1; ++r) a0 += part[(int64_t)r * n + e];
    }
    sh[grp][j] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (grp == 0 && e < n) {
        float s = sh[0][j];
        for (int k = 1; k < kRedG; ++k) s += sh[k][j];
        out[e] = s;
    }
}

__device__ double block_sum(double v, double* sh)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    for (int k = 0; k < nw; ++k) s += sh[k];
    return s;
}

constexpr int kImgParts = 64;   // blocks per image in the per-image reductions

inline unsigned nblk(int64_t n, int bs = 256) { return (unsigned)((n + bs - 1) / bs); }

// part[b][blk] = (sum r^2, sum e^2) over a slice of image b (grid: kImgParts x B)
__global__ __launch_bounds__(256) void k_image_sums(const float* r, const float* e, int64_t npix, double* part)
{
    __shared__ double sh[4];
    const int b = blockIdx.y;
    double sr = 0.0, se = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)kImgParts * 256) {
        const double v = r[(int64_t)b * npix + p];
        sr += v * v;
        if (e) {
            const double u = e[(int64_t)b * npix + p];
            se += u * u;
        }
    }
    sr = block_sum(sr, sh);
    se = block_sum(se, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)b * kImgParts + blockIdx.x) * 2] = sr;
        part[((int64_t)b * kImgParts + blockIdx.x) * 2 + 1] = se;
    }
}

// one thread per image: scale = 1/rms(r); tn = (scale * inv_gain)^2 sum e^2
__global__ void k_image_stats(const double* part, int B, int64_t npix, float* scale, float* tn, float inv_gain)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double sr = 0.0, se = 0.0;
    for (int k = 0; k < kImgParts; ++k) {
        sr += part[((int64_t)b * kImgParts + k) * 2];
        se += part[((int64_t)b * kImgParts + k) * 2 + 1];
    }
    const double s = sr > 0.0 ? 1.0 / sqrt(sr / (double)npix) : 1.0;
    scale[b] = (float)s;
    if (tn) tn[b] = (float)(s * s * inv_gain * inv_gain * se);
}

__global__ __launch_bounds__(256) void k_loss_grad(const float* y, const float* e, const float* scale,
                                                   const float* tn, int B, int64_t npix, float inv_gain,
                                                   float* gy, float* part)
{
    __shared__ double sh[4];
    const int64_t n = (int64_t)B * npix;
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const int b = (int)(i / npix);
        const float d = y[i] - e[i] * (scale[b] * inv_gain);
        gy[i] = 2.f * d / (tn[b] * (float)B);
        acc += (double)d * d / tn[b];
    }
    acc = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = (float)acc;
}

__global__ __launch_bounds__(256) void k_loss_final(const float* part, int nparts, int B, float* loss)
{
    __shared__ double sh[4];
    double s = 0.0;
    for (int k = threadIdx.x; k < nparts; k += 256) s += part[k];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *loss = (float)(s / B);
}

// d = q - r; part[b][blk] = (sum d^2, sum r^2) over a slice of image b (grid: kImgParts x B)
__global__ __launch_bounds__(256) void k_resid_sums(const float* q, const float* r, float* d, int64_t npix,
                                                    double* part)
{
    __shared__ double sh[4];
    const int b = blockIdx.y;
    double sd = 0.0, sr = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)kImgParts * 256) {
        const int64_t i = (int64_t)b * npix + p;
        const float v = q[i] - r[i];
        d[i] = v;
        sd += (double)v * v;
        sr += (double)r[i] * r[i];
    }
    sd = block_sum(sd, sh);
    sr = block_sum(sr, sh);
    if (threadIdx.x == 0) {
        part[((int64_t)b * kImgParts + blockIdx.x) * 2] = sd;
        part[((int64_t)b * kImgParts + blockIdx.x) * 2 + 1] = sr;
    }
}

// one thread per image: rr[b] = sum r^2; lb[b] = sum d^2 / sum r^2
__global__ void k_resid_stats(const double* part, int B, float* rr, float* lb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double sd = 0.0, sr = 0.0;
    for (int k = 0; k < kImgParts; ++k) {
        sd += part[((int64_t)b * kImgParts + k) * 2];
        sr += part[((int64_t)b * kImgParts + k) * 2 + 1];
    }
    rr[b] = (float)sr;
    lb[b] = sr > 0.0 ? (float)(sd / sr) : 0.f;
}

// Energy-norm loss: d = q - r (q = M z); part[b][blk] = (sum z q, sum z r,
// sum e r) over a slice of image b (grid: kImgParts x B)
__global__ __launch_bounds__(256) void k_energy_sums(const float* z, const float* q, const float* r, const float* e,
                                                     float* d, int64_t npix, double* part)
{
    __shared__ double sh[4];
    const int b = blockIdx.y;
    double zq = 0.0, zr = 0.0, er = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < npix; p += (int64_t)kImgParts * 256) {
        const int64_t i = (int64_t)b * npix + p;
        const float qi = q[i], ri = r[i], zi = z[i];
        d[i] = qi - ri;
        zq += (double)zi * qi;
        zr += (double)zi * ri;
        er += (double)e[i] * ri;
    }
    zq = block_sum(zq, sh);
    zr = block_sum(zr, sh);
    er = block_sum(er, sh);
    if (threadIdx.x == 0) {
        double* o = part + ((int64_t)b * kImgParts + blockIdx.x) * 3;
        o[0] = zq;
        o[1] = zr;
        o[2] = er;
    }
}

// one thread per image: er[b] = e^T r = e^T M e; lb[b] = (z - e)^T M (z - e) / e^T M e
//   = (z^T q - 2 z^T r + e^T r) / e^T r
__global__ void k_energy_stats(const double* part, int B, float* er, float* lb)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    double zq = 0.0, zr = 0.0, eer = 0.0;
    for (int k = 0; k < kImgParts; ++k) {
        const double* o = part + ((int64_t)b * kImgParts + k) * 3;
        zq += o[0];
        zr += o[1];
        eer += o[2];
    }
    er[b] = (float)eer;
    lb[b] = eer > 0.0 ? (float)((zq - 2.0 * zr + eer) / eer) : 0.f;
}

// gy = md * 2 gain / (scale[b] * B * rr[b])
__global__ void k_resid_grad(const float* md, const float* scale, const float* rr, int B, int64_t npix, float gain,
                             float* gy)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)B * npix) return;
    const int b = (int)(i / npix);
    gy[i] = rr[b] > 0.f ? md[i] * (2.f * gain / (scale[b] * (float)B * rr[b])) : 0.f;
}

__global__ void k_unscale(const float* y, const float* scale, int64_t npix, int64_t n, float gain, float* z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = y[i] * (gain / scale[i / npix]);
}

__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2,
                       float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

__global__ void k_pack_weights(const float* p, int taps, int cout, int cin, uint16_t* wf, uint16_t* wb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)taps * cout * cin) return;
    const int i = (int)(e % cin), o = (int)((e / cin) % cout), tap = (int)(e / ((int64_t)cin * cout));
    const uint16_t v = (uint16_t)f2bf(p[e]);
    wf[e] = v;
    if (wb) wb[((int64_t)(taps - 1 - tap) * cin + i) * cout + o] = v;
}

__global__ void k_fill(float* p, int64_t n, float v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// out[v][j] = sum_k f[k] in[v][j + k - K/2], zero outside [0, nbins); one
// thread per output
__global__ __launch_bounds__(256) void k_sino_filter(const float* __restrict__ in, int64_t nviews, int nbins,
                                                    const float* __restrict__ f, int K, float* __restrict__ out)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nviews * nbins) return;
    const int64_t v = e / nbins;
    const int j = (int)(e - v * nbins);
    const float* row = in + v * nbins;
    const int h = K / 2;
    float acc = 0.f;
    for (int k = 0; k < K; ++k) {
        const int jj = j + k - h;
        if (jj >= 0 && jj < nbins) acc = fmaf(f[k], row[jj], acc);
    }
    out[e] = acc;
}

// z += mu * r
__global__ void k_add_scaled(int64_t n, float mu, const float* __restrict__ r, float* __restrict__ z)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = fmaf(mu, r[i], z[i]);
}

// ------------------------------------------------------------- solver kernels
__global__ void k_reg(const float* c, float* out, int nx, int ny, float lam, int accumulate)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= (int64_t)nx * ny) return;
    const int i = (int)(k % nx), j = (int)(k / nx);
    const float c0 = c[k];
    float v = 0.f;
    if (i > 0) v += c0 - c[k - 1];
    if (i < nx - 1) v += c0 - c[k + 1];
    if (j > 0) v += c0 - c[k - nx];
    if (j < ny - 1) v += c0 - c[k + nx];
    out[k] = (accumulate ? out[k] : 0.f) + lam * v;
}

constexpr int kDotParts = 512;   // k_dots_final reduces up to kMaxVecs rows of this many partials

__global__ __launch_bounds__(256) void k_dots(int64_t n, const float* a0, const float* b0, const float* a1,
                                              const float* b1, const float* a2, const float* b2, double* part)
{
    __shared__ double sh[4];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        if (a0) s0 += (double)a0[i] * b0[i];
        if (a1) s1 += (double)a1[i] * b1[i];
        if (a2) s2 += (double)a2[i] * b2[i];
    }
    s0 = block_sum(s0, sh);
    s1 = block_sum(s1, sh);
    s2 = block_sum(s2, sh);
    if (threadIdx.x == 0) {
        part[blockIdx.x] = s0;
        part[kDotParts + blockIdx.x] = s1;
        part[2 * kDotParts + blockIdx.x] = s2;
    }
}

__global__ __launch_bounds__(256) void k_dots_final(const double* part, int nk, double* slots, int slot0)
{
    __shared__ double sh[4];
    for (int k = 0; k < nk; ++k) {
        double s = 0.0;
        for (int i = threadIdx.x; i < kDotParts; i += 256) s += part[k * kDotParts + i];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) slots[slot0 + k] = s;
    }
}

__global__ void k_axpy2(int64_t n, const double* slots, int num, int den, int sign, const float* x,
                        const float* d, float* y, const float* x2, const float* d2, float* y2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float al = (float)(sign * slots[num] / slots[den]);
    y[i] = x[i] + al * d[i];
    if (y2) y2[i] = x2[i] - al * d2[i];
}

__global__ void k_direction(int64_t n, const double* slots, int a, int b, int c, const float* z, const float* p,
                            float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (c < 0) {
        out[i] = z[i];   // first step: no previous direction is read
        return;
    }
    const float beta = (float)((slots[a] - (b >= 0 ? slots[b] : 0.0)) / slots[c]);
    out[i] = z[i] + beta * p[i];
}

__global__ void k_flip(const uint16_t* w, int taps, int cout, int cin, uint16_t* wb)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)taps * cout * cin) return;
    const int i = (int)(e % cin), o = (int)((e / cin) % cout), tap = (int)(e / ((int64_t)cin * cout));
    wb[((int64_t)(taps - 1 - tap) * cin + i) * cout + o] = w[e];
}

__global__ void k_copy_slot(double* slots, int dst, int src) { slots[dst] = slots[src]; }

// part[j][block] = partial sums of <x, y_j>, j < k
__global__ __launch_bounds__(256) void k_dots_multi(int64_t n, const float* x, VecList ys, int k, double* part)
{
    __shared__ double sh[4];
    double acc[kMaxVecs];
#pragma unroll
    for (int j = 0; j < kMaxVecs; ++j) acc[j] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double xv = x[i];
#pragma unroll
        for (int j = 0; j < kMaxVecs; ++j)
            if (j < k) acc[j] += xv * ys.v[j][i];
    }
    for (int j = 0; j < k; ++j) {
        const double s = block_sum(acc[j], sh);
        if (threadIdx.x == 0) part[j * kDotParts + blockIdx.x] = s;
    }
}

// out = z - sum_j (slots[a + j] / slots[b + j]) ps_j
__global__ void k_orth(int64_t n, const double* slots, int a, int b, int k, const float* z, VecList ps, float* out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = z[i];
    for (int j = 0; j < k; ++j) v -= (float)(slots[a + j] / slots[b + j]) * ps.v[j][i];
    out[i] = v;
}



}  // namespace

// ------------------------------------------------------------------ launchers
// tiles x images x output-channel blocks of the unsplit launch, and the split
// that brings it to about 512 workgroups (at most one chunk of 32 input
// channels per split)
static void conv_shape(int B, int H, int W, int cin, int cout, bool* wide, int* ksplit)
{
    const int64_t ntiles = (int64_t)((W + kTW - 1) / kTW) * ((H + kTR - 1) / kTR);
    *wide = cout % 64 == 0 && ntiles * B * (cout / 64) >= 512;
    const int64_t wgs = ntiles * B * (cout / (*wide ? 64 : 32));
    int k = 1;
    while (wgs * k * 2 <= 512 && k * 2 <= cin / 32) k *= 2;
    *ksplit = k;
}

int64_t conv3x3_ws_floats(int B, int H, int W, int cin, int cout)
{
    bool wide;
    int k;
    conv_shape(B, H, W, cin, cout, &wide, &k);
    return k > 1 ? (int64_t)k * B * H * W * cout : 0;
}

hipError_t conv3x3(const ConvArgs& a0, bool f32_out, float* ws, int64_t ws_floats, hipStream_t s)
{
    if (a0.cin % 32 || a0.cout % 32 || a0.B <= 0 || a0.H <= 0 || a0.W <= 0 || a0.B > 65535) return hipErrorInvalidValue;
    ConvArgs a = a0;
    const int ntiles = ((a.W + kTW - 1) / kTW) * ((a.H + kTR - 1) / kTR);
    bool wide;
    int k;
    conv_shape(a.B, a.H, a.W, a.cin, a.cout, &wide, &k);
    if (k > 1 && (!ws || (int64_t)k * a.B * a.H * a.W * a.cout > ws_floats)) k = 1;
    a.ksplit = k;
    a.kpart = k > 1 ? ws : nullptr;
    const dim3 grid(ntiles, a.B, (a.cout / (wide ? 64 : 32)) * k);
    if (a.in_mode == kConvPool) {
        if (f32_out) return hipErrorInvalidValue;
        if (wide) hipLaunchKernelGGL((k_conv3x3<64, false, kConvPool>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<32, false, kConvPool>), grid, dim3(256), 0, s, a);
    } else if (a.in_mode == kConvUpcat) {
        if (f32_out || (a.cin / 2) % 32 || !a.x2.p) return hipErrorInvalidValue;
        if (wide) hipLaunchKernelGGL((k_conv3x3<64, false, kConvUpcat>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<32, false, kConvUpcat>), grid, dim3(256), 0, s, a);
    } else if (a.in_mode != kConvPlain) {
        return hipErrorInvalidValue;
    } else if (wide) {
        if (f32_out) hipLaunchKernelGGL((k_conv3x3<64, true, kConvPlain>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<64, false, kConvPlain>), grid, dim3(256), 0, s, a);
    } else {
        if (f32_out) hipLaunchKernelGGL((k_conv3x3<32, true, kConvPlain>), grid, dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k_conv3x3<32, false, kConvPlain>), grid, dim3(256), 0, s, a);
    }
    if (k > 1) {
        const int64_t n = (int64_t)a.B * a.H * a.W * (a.cout / 4);
        hipLaunchKernelGGL(k_conv_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a, f32_out ? 1 : 0);
    }
    return hipGetLastError();
}

int wgrad_rows(int B, int H, int W, int cin, int cout)
{
    // aim for ~512 workgroups: regions x (cout/32) x (cin/32)
    const int64_t tiles = (int64_t)(cout / 32) * (cin / 32) * B * ((W + 63) / 64);
    int64_t want = 512 / (tiles > 0 ? tiles : 1);
    if (want < 1) want = 1;
    int rows = (int)((H + want - 1) / want);
    rows = (rows + 1) & ~1;
    if (rows < 2) rows = 2;
    return rows;
}

int64_t wgrad_regions(int B, int H, int W, int rows)
{
    return (int64_t)B * ((H + rows - 1) / rows) * ((W + 63) / 64);
}

hipError_t conv3x3_wgrad(const WgradArgs& a, int* n_regions, hipStream_t s)
{
    if (a.cin % 32 || a.cout % 32 || a.rows < 2 || (a.rows & 1)) return hipErrorInvalidValue;
    const int64_t nreg = wgrad_regions(a.B, a.H, a.W, a.rows);
    *n_regions = (int)nreg;
    hipLaunchKernelGGL(k_wgrad, dim3((unsigned)nreg, (a.cout / 32) * (a.cin / 32)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t conv_in(const float* x, const float* scale, const uint16_t* w, View y, int c, int B, int H, int W,
                   bool relu, hipStream_t s)
{
    if (c % 8 || c > 256) return hipErrorInvalidValue;
    const int64_t n = (int64_t)B * H * W * (c / 8);
    hipLaunchKernelGGL(k_conv_in, dim3(nblk(n)), dim3(256), 0, s, x, scale, w, y, c, B, H, W, relu ? 1 : 0);
    return hipGetLastError();
}

// pixels per workgroup of the 1-channel and 1x1 layers' weight gradients:
// about 4096 workgroups (at least 64 pixels each), so that the loads of many
// pixels are in flight
int per_block_pixels(int64_t npix) { return (int)((npix + 4095) / 4096 < 64 ? 64 : (npix + 4095) / 4096); }

hipError_t conv_in_wgrad(const float* x, const float* scale, CView g, int c, int B, int H, int W, float* part,
                         int* n_regions, hipStream_t s)
{
    if (c <= 0 || 256 % c) return hipErrorInvalidValue;
    const int64_t npix = (int64_t)B * H * W;
    const int per = per_block_pixels(npix);
    const int nb = (int)((npix + per - 1) / per);
    *n_regions = nb;
    hipLaunchKernelGGL(k_conv_in_wgrad, dim3(nb), dim3(256), 0, s, x, scale, g, c, B, H, W, per, part);
    return hipGetLastError();
}

hipError_t conv_out(CView d, const uint16_t* w, int c, float* y, int npix, hipStream_t s, const float* scale,
                    float gain, int64_t img_npix)
{
    if (scale && img_npix < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_conv_out, dim3(nblk(npix)), dim3(256), 0, s, d, w, c, y, (int64_t)npix, scale, gain,
                       img_npix);
    return hipGetLastError();
}

hipError_t conv_out_bwd(CView d, const uint16_t* w, const float* gy, int c, View gd, int npix, bool mask,
                        hipStream_t s)
{
    const int64_t n = (int64_t)npix * (c / 8);
    hipLaunchKernelGGL(k_conv_out_bwd, dim3(nblk(n)), dim3(256), 0, s, d, w, gy, c, gd, (int64_t)npix, mask ? 1 : 0);
    return hipGetLastError();
}

hipError_t conv_out_wgrad(CView d, const float* gy, int c, int npix, float* part, int* n_regions, hipStream_t s)
{
    if (c <= 0 || 256 % c) return hipErrorInvalidValue;
    const int per = per_block_pixels(npix);
    const int nb = (int)((npix + per - 1) / per);
    *n_regions = nb;
    hipLaunchKernelGGL(k_conv_out_wgrad, dim3(nb), dim3(256), 0, s, d, gy, c, (int64_t)npix, per, part);
    return hipGetLastError();
}

hipError_t avgpool2(CView x, View y, int c, int B, int H, int W, hipStream_t s)
{
    const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (c / 8);
    hipLaunchKernelGGL(k_avgpool2, dim3(nblk(n)), dim3(256), 0, s, x, y, c, B, H, W);
    return hipGetLastError();
}

hipError_t avgpool2_T_add(CView gc, View g, CView e, int c, int B, int H, int W, hipStream_t s)
{
    const int64_t n = (int64_t)B * H * W * (c / 8);
    hipLaunchKernelGGL(k_avgpool2_T_add, dim3(nblk(n)), dim3(256), 0, s, gc, g, e, c, B, H, W);
    return hipGetLastError();
}

hipError_t upsample2(CView x, View y, int c, int B, int H, int W, hipStream_t s)
{
    const int64_t n = (int64_t)B * H * W * (c / 8);
    hipLaunchKernelGGL(k_upsample2, dim3(nblk(n)), dim3(256), 0, s, x, y, c, B, H, W);
    return hipGetLastError();
}

hipError_t upsample2_T(CView g, View y, int c, int B, int H, int W, hipStream_t s)
{
    const int64_t n = (int64_t)B * (H / 2) * (W / 2) * (c / 8);
    hipLaunchKernelGGL(k_upsample2_T, dim3(nblk(n)), dim3(256), 0, s, g, y, c, B, H, W);
    return hipGetLastError();
}

hipError_t reduce_parts(const float* part, int nreg, int64_t n, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)((n + kRedE - 1) / kRedE)), dim3(256), 0, s, part, nreg, n, out);
    return hipGetLastError();
}

int image_parts() { return kImgParts; }

hipError_t image_stats(const float* r, const float* e, int B, int64_t npix, float gain, float* scale, float* tn,
                       double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_image_sums, dim3(kImgParts, B), dim3(256), 0, s, r, e, npix, part);
    hipLaunchKernelGGL(k_image_stats, dim3(nblk(B, 64)), dim3(64), 0, s, part, B, npix, scale, tn, 1.f / gain);
    return hipGetLastError();
}

hipError_t loss_grad(const float* y, const float* e, const float* scale, const float* tn, int B, int64_t npix,
                     float gain, float* gy, float* part, float* loss, hipStream_t s)
{
    const int nb = 256;
    hipLaunchKernelGGL(k_loss_grad, dim3(nb), dim3(256), 0, s, y, e, scale, tn, B, npix, 1.f / gain, gy, part);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, part, nb, B, loss);
    return hipGetLastError();
}

hipError_t resid_stats(const float* q, const float* r, float* d, int B, int64_t npix, float* rr, float* lb,
                       float* loss, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_resid_sums, dim3(kImgParts, B), dim3(256), 0, s, q, r, d, npix, part);
    hipLaunchKernelGGL(k_resid_stats, dim3(nblk(B, 64)), dim3(64), 0, s, part, B, rr, lb);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, lb, B, B, loss);
    return hipGetLastError();
}

hipError_t energy_stats(const float* z, const float* q, const float* r, const float* e, float* d, int B,
                        int64_t npix, float* er, float* lb, float* loss, double* part, hipStream_t s)
{
    hipLaunchKernelGGL(k_energy_sums, dim3(kImgParts, B), dim3(256), 0, s, z, q, r, e, d, npix, part);
    hipLaunchKernelGGL(k_energy_stats, dim3(nblk(B, 64)), dim3(64), 0, s, part, B, er, lb);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, s, lb, B, B, loss);
    return hipGetLastError();
}

hipError_t resid_grad(const float* md, const float* scale, const float* rr, int B, int64_t npix, float gain,
                      float* gy, hipStream_t s)
{
    const int64_t n = (int64_t)B * npix;
    hipLaunchKernelGGL(k_resid_grad, dim3(nblk(n)), dim3(256), 0, s, md, scale, rr, B, npix, gain, gy);
    return hipGetLastError();
}

hipError_t unscale(const float* y, const float* scale, int B, int64_t npix, float gain, float* z, hipStream_t s)
{
    const int64_t n = (int64_t)B * npix;
    hipLaunchKernelGGL(k_unscale, dim3(nblk(n)), dim3(256), 0, s, y, scale, npix, n, gain, z);
    return hipGetLastError();
}

hipError_t adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t pack_weights(const float* p, int taps, int cout, int cin, uint16_t* wf, uint16_t* wb, hipStream_t s)
{
    const int64_t n = (int64_t)taps * cout * cin;
    hipLaunchKernelGGL(k_pack_weights, dim3(nblk(n)), dim3(256), 0, s, p, taps, cout, cin, wf, wb);
    return hipGetLastError();
}

hipError_t fill_f32(float* p, int64_t n, float v, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill, dim3(nblk(n)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t sino_filter(const float* in, int64_t nviews, int nbins, const float* f, int K, float* out, hipStream_t s)
{
    const int64_t n = nviews * nbins;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sino_filter, dim3(nblk(n)), dim3(256), 0, s, in, nviews, nbins, f, K, out);
    return hipGetLastError();
}

hipError_t add_scaled(int64_t n, float mu, const float* r, float* z, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_add_scaled, dim3(nblk(n)), dim3(256), 0, s, n, mu, r, z);
    return hipGetLastError();
}

hipError_t reg_apply(const float* c, float* out, int nx, int ny, float lam, bool accumulate, hipStream_t s)
{
    hipLaunchKernelGGL(k_reg, dim3(nblk((int64_t)nx * ny)), dim3(256), 0, s, c, out, nx, ny, lam, accumulate ? 1 : 0);
    return hipGetLastError();
}

int dots_parts() { return kDotParts; }

hipError_t dots(int64_t n, const float* a0, const float* b0, const float* a1, const float* b1, const float* a2,
                const float* b2, double* part, double* slots, int slot0, hipStream_t s)
{
    const int nk = a2 ? 3 : (a1 ? 2 : 1);
    hipLaunchKernelGGL(k_dots, dim3(kDotParts), dim3(256), 0, s, n, a0, b0, a1, b1, a2, b2, part);
    hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, s, part, nk, slots, slot0);
    return hipGetLastError();
}

hipError_t axpy2(int64_t n, const double* slots, int num, int den, int sign_num, const float* x, const float* d,
                 float* y, const float* x2, const float* d2, float* y2, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy2, dim3(nblk(n)), dim3(256), 0, s, n, slots, num, den, sign_num, x, d, y, x2, d2, y2);
    return hipGetLastError();
}

hipError_t direction(int64_t n, const double* slots, int a, int b, int c, const float* z, const float* p, float* out,
                     hipStream_t s)
{
    hipLaunchKernelGGL(k_direction, dim3(nblk(n)), dim3(256), 0, s, n, slots, a, b, c, z, p, out);
    return hipGetLastError();
}

hipError_t flip_weights(const uint16_t* w, int taps, int cout, int cin, uint16_t* wb, hipStream_t s)
{
    const int64_t n = (int64_t)taps * cout * cin;
    hipLaunchKernelGGL(k_flip, dim3(nblk(n)), dim3(256), 0, s, w, taps, cout, cin, wb);
    return hipGetLastError();
}

hipError_t dots_multi(int64_t n, const float* x, const VecList& ys, int k, double* part, double* slots, int slot0,
                      hipStream_t s)
{
    if (k < 1 || k > kMaxVecs) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_dots_multi, dim3(kDotParts), dim3(256), 0, s, n, x, ys, k, part);
    hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(256), 0, s, part, k, slots, slot0);
    return hipGetLastError();
}

hipError_t orth(int64_t n, const double* slots, int a, int b, int k, const float* z, const VecList& ps, float* out,
                hipStream_t s)
{
    if (k < 0 || k > kMaxVecs) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_orth, dim3(nblk(n)), dim3(256), 0, s, n, slots, a, b, k, z, ps, out);
    return hipGetLastError();
}

hipError_t copy_slot(double* slots, int dst, int src, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_slot, dim3(1), dim3(1), 0, s, slots, dst, src);
    return hipGetLastError();
}

}  // namespace xrl
