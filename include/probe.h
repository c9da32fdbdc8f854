/*
 * probe.h -- attainable peaks of the running GPU, measured by short
 * microbenchmarks, as roofline denominators beside the published figures
 * (MI355X: FP32 vector 157.3 TFLOP/s with packed instructions, 78.6 without;
 * BF16 matrix 2.5 PFLOP/s dense; HBM3E 8 TB/s); and an elementwise probe of
 * the rollout kernel's own sine and cosine for accuracy tests.
 *
 *  probe_fp32_fma   every lane runs 8 independent fused multiply-add chains
 *                   of `iters` links, compiled like the simulator's kernels
 *                   (packed FP32 disabled), `blocks` workgroups of 256
 *                   threads; TFLOP/s with FMA = 2 flops.
 *  probe_bf16_mfma  every wave issues v_mfma_f32_16x16x32_bf16 (the
 *                   surrogate's product instruction) on 4 independent
 *                   accumulators, `iters` rounds, `blocks` workgroups of 256
 *                   threads; TFLOP/s with 16 x 16 x 32 x 2 flops per
 *                   instruction.
 *  probe_copy       a plain vector copy kernel (16 bytes per lane per
 *                   access, grid-stride) of `bytes` from src to dst; GB/s
 *                   counting the bytes read plus the bytes written.
 *  probe_sincos     sn[i], cs[i] = the sine and cosine the rollout kernel
 *                   uses for joint angles and CPG phases (range reduction by
 *                   pi/2, Taylor series on |r| <= pi/4), of x[i] in radians,
 *                   i < n (1 <= n <= 2^31); x, sn, cs are DEVICE float
 *                   arrays of n owned by the caller.  Asynchronous on the
 *                   stream: returns after the launch, no timing.
 *
 * Conventions: `sink`, `src` and `dst` are DEVICE memory owned by the
 * caller (sink: blocks * 256 floats, written so the compiler keeps the
 * arithmetic; src and dst: `bytes` each, a multiple of 16, not
 * overlapping); nothing is allocated.  Each call records HIP events around
 * one launch on the given stream (void*, NULL = null stream), waits for the
 * second, and writes the rate to *result (host).  Return value: PROBE_OK or a
 * negative PROBE_E_* code, with a message from probe_last_error() (per host
 * thread).
 */
#ifndef PROBE_H_
#define PROBE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PROBE_OK 0
#define PROBE_E_INVALID (-1) /* bad argument (nothing was launched) */
#define PROBE_E_DEVICE (-2)  /* HIP error                             */

int probe_fp32_fma(float* sink, int32_t blocks, int32_t iters, void* stream, double* tflops);
int probe_bf16_mfma(float* sink, int32_t blocks, int32_t iters, void* stream, double* tflops);
int probe_copy(const void* src, void* dst, size_t bytes, void* stream, double* gbs);
int probe_sincos(const float* x, float* sn, float* cs, int64_t n, void* stream);

const char* probe_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PROBE_H_ */
