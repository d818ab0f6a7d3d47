/*
 * tt_probe.h -- calibration kernels used to read hardware counters and
 * ceilings next to the channel kernels (not part of the channel path).
 */
#ifndef TT_PROBE_H
#define TT_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Copies bytes (a multiple of 16) from src to dst, both device pointers, on
 * hip_stream (hipStream_t or NULL).  Used to calibrate HBM byte counters:
 * it reads and writes exactly `bytes` each.  Returns 0 or a HIP error code. */
int32_t tt_probe_copy(void *dst, const void *src, int64_t bytes, void *hip_stream);

/* Runs `blocks` workgroups of 256 threads, each thread doing `iters` x 64
 * independent FP32 fused multiply-adds (unpacked v_fma_f32) and writing one
 * float to out[blocks * 256].  Measures the vector-ALU FMA ceiling.
 * Returns 0 or a HIP error code. */
int32_t tt_probe_fma(float *out, int32_t blocks, int32_t iters, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
