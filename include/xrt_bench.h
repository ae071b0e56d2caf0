/* Measurement support of libxrt.so (not part of the transform).
 *
 * xrt_calib_valu launches `blocks` workgroups of 256 threads on `stream`;
 * every thread runs `iters` iterations of 64 dependent-in-8-chains vector
 * operations: mode 0 FP32 fused multiply-add (v_fma_f32), mode 1 32-bit
 * integer add (v_add_u32), mode 2 FP64 fused multiply-add (v_fma_f64), and writes
 * one float per thread to out [blocks * 256] (device memory, caller-owned).
 * A wave therefore issues 64 * iters VALU instructions of the chosen kind
 * plus a fixed prologue and epilogue.  Used to calibrate the VALU issue rate
 * and the SQ/GRBM counters against which the transform kernels' busy
 * fractions are reported.  Returns 0, -1 for invalid arguments, -5 for a
 * launch failure.  No allocation, no synchronisation.
 *
 * xrt_calib_lds launches `blocks` workgroups of 256 threads on `stream`;
 * every thread makes `iters` x 16 32-bit integer atomic adds into a
 * 4096-word LDS array of its workgroup, at 16 addresses fixed per thread by
 * `pattern` (0..7, from the lane within the wave: consecutive words, strides
 * 2, 32, 64 and 65, one word per instruction for all lanes, lanes in pairs
 * on one word, and hashed addresses; 8 and 9: 64-bit atomic adds at
 * consecutive and at hashed doublewords), then writes one float per thread to
 * out [blocks * 256] (device memory, caller-owned).  Used to measure the
 * LDS cost of an atomic with and without bank conflicts (time and the
 * SQ_LDS_BANK_CONFLICT counter).  Same return codes as xrt_calib_valu. */
#ifndef XRT_BENCH_H
#define XRT_BENCH_H

#ifdef __cplusplus
extern "C" {
#endif

int xrt_calib_valu(int mode, int iters, int blocks, float* out, void* stream);
int xrt_calib_lds(int pattern, int iters, int blocks, float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif
