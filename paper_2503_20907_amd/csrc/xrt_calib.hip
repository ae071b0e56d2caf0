// Measurement support: a kernel with a known number of vector ALU
// instructions, to calibrate the issue rate of the VALU (wave instructions
// per cycle per SIMD) and to check what the SQ_INSTS_VALU,
// SQ_ACTIVE_INST_VALU and GRBM_GUI_ACTIVE counters report, so that the
// counters taken on the transform kernels can be turned into a busy
// fraction against a measured ceiling.
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
