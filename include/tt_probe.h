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

/* HBM ceilings: kind 0 reads `bytes` from src (writing one 16-byte word per
 * workgroup to dst, which must hold `blocks` of them), kind 1 writes `bytes`
 * to dst, kind 2 copies `bytes` from src to dst.  `blocks` workgroups of 256
 * threads stride through the buffers, each thread keeping four 16-byte
 * accesses in flight; nontemporal != 0 marks the stores non-temporal.  bytes
 * a multiple of 16 (>= 16), blocks in 1 .. 2^20, device pointers, hip_stream
 * a hipStream_t or NULL.  Returns 0 or a HIP error code (hipErrorInvalidValue
 * for bad arguments, nothing launched). */
int32_t tt_probe_stream(int32_t kind, void *dst, const void *src, int64_t bytes, int32_t blocks,
                        int32_t nontemporal, void *hip_stream);

/* Write ceiling of a scattered output pattern: `bytes` (a multiple of 8192)
 * written as 8 KiB chunks, each by one workgroup whose lanes store two
 * 16-byte words 32 bytes apart; chunk q lies in stream q mod `streams` (the
 * buffer cut into `streams` equal slices) at position q div `streams`, and
 * `blocks` workgroups take chunks q = blockIdx, blockIdx + blocks, ...  A
 * chunk count not divisible by `streams` leaves the remainder unwritten.
 * streams in 1 .. bytes / 8192.  Returns 0 or a HIP error code. */
int32_t tt_probe_chunked_write(void *dst, int64_t bytes, int32_t streams, int32_t blocks, int32_t nontemporal,
                               void *hip_stream);

/* Runs `blocks` workgroups of 256 threads, each thread doing `iters` x 64
 * independent FP32 fused multiply-adds (unpacked v_fma_f32) and writing one
 * float to out[blocks * 256].  Measures the vector-ALU FMA ceiling.
 * Returns 0 or a HIP error code. */
int32_t tt_probe_fma(float *out, int32_t blocks, int32_t iters, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
