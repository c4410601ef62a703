/*
 * gfc_microbench.h -- rate probes of the device the renderer runs on, for
 * the denominators of its roofline: how fast the vector ALUs issue FP32
 * FMAs, how fast they issue v_exp_f32 alone and when it is interleaved with
 * FMAs (the exponential is where the method spends its time, Section 3 of
 * Lang 2020), and how fast HBM takes a streamed write and a copy.
 *
 * Every probe runs on the current HIP device and on `hip_stream`: one
 * untimed launch, then `reps` timed launches bracketed by HIP events on that
 * stream; it returns the best rate of the timed launches.  The calls
 * synchronise the stream.  They allocate nothing: device buffers come from
 * the caller.  Return value: 0, or a negative hipError_t value when a launch
 * or an event call fails (no probe result is written then).
 */
#ifndef GFC_MICROBENCH_H_
#define GFC_MICROBENCH_H_

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* FP32 fused multiply-adds (v_fma_f32, no packed forms), 16 independent
 * dependency chains per lane, enough wavefronts to fill every SIMD.  sink:
 * device, >= 4 bytes (written only on an impossible result, which keeps
 * the arithmetic live).  out: lane-FMAs per second (FLOP/s = 2x). */
int gfc_mb_fma(int reps, float* sink, void* hip_stream, double* lane_fma_per_s);

/* v_exp_f32 alone: 16 independent chains x <- exp2(-x) per lane.  out:
 * lane-exponentials per second. */
int gfc_mb_exp(int reps, float* sink, void* hip_stream, double* lane_exp_per_s);

/* v_exp_f32 interleaved with independent FMAs: per step, one exponential
 * chain x <- exp2(-x) and fma_per_exp FMAs on other accumulators (0..8), in
 * 8 independent groups per lane.  out: lane-exponentials per second and
 * lane-FMAs per second of the mixed stream. */
int gfc_mb_exp_fma(int fma_per_exp, int reps, float* sink, void* hip_stream, double* lane_exp_per_s,
                   double* lane_fma_per_s);

/* Streamed (non-temporal) 16-byte writes of `bytes` bytes (a multiple of
 * 16) to dst (device).  out: bytes written per second. */
int gfc_mb_hbm_write(float* dst, size_t bytes, int reps, void* hip_stream, double* bytes_per_s);

/* Copy of `bytes` bytes (a multiple of 16) from src to dst (device, not
 * overlapping), 16-byte loads and streamed stores.  out: bytes moved per
 * second, counting the read and the write (2 x bytes per launch). */
int gfc_mb_hbm_copy(float* dst, const float* src, size_t bytes, int reps, void* hip_stream,
                    double* bytes_per_s);

#ifdef __cplusplus
}
#endif

#endif /* GFC_MICROBENCH_H_ */
