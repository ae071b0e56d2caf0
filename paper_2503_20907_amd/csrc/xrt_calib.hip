// Measurement support: a kernel with a known number of vector ALU
// instructions, to calibrate the issue rate of the VALU (wave instructions
// per cycle per SIMD) and to check what the SQ_INSTS_VALU,
// SQ_ACTIVE_INST_VALU and GRBM_GUI_ACTIVE counters report, so that the
// counters taken on the transform kernels can be turned into a busy
// fraction against a measured ceiling; and a kernel with a known number of
// LDS integer atomics per wave in chosen address patterns, to measure what
// an atomic costs the LDS with and without bank conflicts.
//
// Every thread runs 8 dependency chains of one operation (for integers the
// chains feed each other, so that the compiler cannot fold them); the
// loop body holds 8 x 8 = 64 of them, its counter lives in scalar
// registers, so each wave issues 64 VALU instructions per iteration (plus a
// fixed prologue and epilogue of a few dozen).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xrt_bench.h"

namespace {

template <int MODE>
__global__ void __launch_bounds__(256) k_calib_valu(float* out, int iters)
{
    const int tid = blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (MODE == 0) {
        float a[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = 1.0f + 1e-3f * (float)(tid + c);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) a[c] = fmaf(a[c], 0.999999f, 1e-7f);
        }
        float s = 0.f;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += a[c];
        out[tid] = s;
    } else if constexpr (MODE == 1) {
        uint32_t a[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = (uint32_t)(tid * 8 + c);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) a[c] += a[(c + 1) & 7];
        }
        uint32_t s = 0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s ^= a[c];
        out[tid] = (float)s;
    } else {
        double a[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) a[c] = 1.0 + 1e-3 * (double)(tid + c);
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < 8; ++c) a[c] = fma(a[c], 0.999999, 1e-7);
        }
        double s = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) s += a[c];
        out[tid] = (float)s;
    }
}

// Every thread makes iters x 16 ds_add_u32 into a 4096-word LDS array at
// 16 fixed addresses chosen by `pattern` from its lane l (0..63), wave w
// and slot u (0..15):
//   0: 64 w + l (consecutive words)       1: 2 l + 128 u (stride 2)
//   2: 32 l + u (stride 32)               3: 64 u (one word for all lanes)
//   4: a hash of (block, w, l, u)          5: 64 l + u (stride 64)
//   6: l / 2 + 64 u (lanes in pairs on one word)
//   7: 65 l + u (stride 65)
// Patterns 8 and 9 make 64-bit atomic adds (ds_add_u64) into the same array
// read as 2048 doublewords: 8 at 64 w + l + 256 u (consecutive), 9 at hashed
// doublewords.
// The addresses are formed before the loop, whose body is 16 atomics.
template <int P>
__device__ inline uint32_t lds_addr(uint32_t b, uint32_t w, uint32_t l, uint32_t u)
{
    if constexpr (P == 0) return (64u * w + l + 256u * u) & 4095u;
    else if constexpr (P == 1) return (2u * l + 128u * u) & 4095u;
    else if constexpr (P == 2) return (32u * l + u) & 4095u;
    else if constexpr (P == 3) return 64u * u;
    else if constexpr (P == 4) {
        uint32_t h = (b * 0x9E3779B1u) ^ (w * 0x85EBCA77u) ^ (l * 0xC2B2AE3Du) ^ (u * 0x27D4EB2Fu);
        h ^= h >> 15;
        h *= 0x2C1B3C6Du;
        h ^= h >> 12;
        return h & 4095u;
    } else if constexpr (P == 5) return (64u * l + u) & 4095u;
    else if constexpr (P == 6) return (l / 2u + 64u * u) & 4095u;
    else return (65u * l + u) & 4095u;
}

template <int P>
__global__ void __launch_bounds__(256) k_calib_lds(float* out, int iters)
{
    __shared__ unsigned long long acc[2048];
    for (int e = threadIdx.x; e < 2048; e += 256) acc[e] = 0ull;
    __syncthreads();
    const uint32_t l = threadIdx.x & 63u, w = threadIdx.x >> 6;
    uint32_t a[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        if constexpr (P < 8) a[u] = lds_addr<P>(blockIdx.x, w, l, (uint32_t)u);
        else a[u] = lds_addr<P == 8 ? 0 : 4>(blockIdx.x, w, l, (uint32_t)u) & 2047u;
    }
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            if constexpr (P < 8) atomicAdd((unsigned int*)acc + a[u], 1u);
            else atomicAdd(acc + a[u], 1ull);
        }
    }
    __syncthreads();
    out[blockIdx.x * 256 + threadIdx.x] = (float)acc[threadIdx.x];
}

}  // namespace

extern "C" int xrt_calib_valu(int mode, int iters, int blocks, float* out, void* stream)
{
    if (!out || iters < 1 || blocks < 1 || mode < 0 || mode > 2) return -1;
    hipStream_t s = (hipStream_t)stream;
    switch (mode) {
    case 0: hipLaunchKernelGGL(k_calib_valu<0>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(k_calib_valu<1>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    default: hipLaunchKernelGGL(k_calib_valu<2>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

extern "C" int xrt_calib_lds(int pattern, int iters, int blocks, float* out, void* stream)
{
    if (!out || iters < 1 || blocks < 1 || pattern < 0 || pattern > 9) return -1;
    hipStream_t s = (hipStream_t)stream;
    switch (pattern) {
    case 0: hipLaunchKernelGGL(k_calib_lds<0>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 1: hipLaunchKernelGGL(k_calib_lds<1>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 2: hipLaunchKernelGGL(k_calib_lds<2>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 3: hipLaunchKernelGGL(k_calib_lds<3>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 4: hipLaunchKernelGGL(k_calib_lds<4>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 5: hipLaunchKernelGGL(k_calib_lds<5>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 6: hipLaunchKernelGGL(k_calib_lds<6>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 7: hipLaunchKernelGGL(k_calib_lds<7>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    case 8: hipLaunchKernelGGL(k_calib_lds<8>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    default: hipLaunchKernelGGL(k_calib_lds<9>, dim3(blocks), dim3(256), 0, s, out, iters); break;
    }
    return hipGetLastError() == hipSuccess ? 0 : -5;
}
