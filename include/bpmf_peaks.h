/*
 * bpmf_peaks.h -- micro-benchmarks that measure the peaks of the device the
 * calling thread has current, so that the sweep's roofline can be stated
 * against measured rates as well as against the spec sheet.
 *
 * The roofline of a row update (Sec. II: every row is a few K x K matrix and
 * vector operations plus one K x K factorisation, fed by the rows of the
 * other factor that its ratings name) is bounded by the HBM rate, the rate of
 * random K-wide row gathers from the other factor (which depends on whether
 * that factor fits in L2, in the Infinity Cache or only in HBM), and the
 * FP32 / BF16 matrix-core and vector rates.  Each call below measures one of
 * these with a kernel of its own.
 *
 * Conventions: every call uses the current HIP device and a private stream,
 * allocates what it needs with hipMalloc and frees it before returning,
 * launches one untimed warm-up and then `reps` timed launches (HIP events
 * around each), and returns the best of them.  Returns BPMF_OK (0),
 * BPMF_E_INVAL (-1) for a bad argument, BPMF_E_NOMEM (-4) when an allocation
 * fails or BPMF_E_DEVICE (-5) for any other HIP error.  No context is
 * involved; the calls may run while no context exists.
 */
#ifndef BPMF_PEAKS_H
#define BPMF_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Kinds of bpmf_peak_compute. */
#define BPMF_PEAK_FP32_VALU 0 /* v_fma_f32 (unpacked: the library is built without packed FP32) */
#define BPMF_PEAK_FP32_MFMA 1 /* v_mfma_f32_16x16x4_f32 */
#define BPMF_PEAK_BF16_MFMA 2 /* v_mfma_f32_16x16x32_bf16 */
#define BPMF_PEAK_FP64_MFMA 3 /* v_mfma_f64_16x16x4_f64 */

/* Stream triad a = b + s c over three device arrays of `bytes_per_array`
 * bytes each (a multiple of 16, at least 1 MiB).  *gbs = 3 * bytes_per_array
 * / time, in GB/s (1e9 B/s). */
int bpmf_peak_triad(int64_t bytes_per_array, int32_t reps, double *gbs);

/* Dense arithmetic rate of one instruction kind (BPMF_PEAK_*), every CU
 * busy, independent accumulators per wavefront; *tflops in TFLOP/s (an FMA
 * counts two FLOP). */
int bpmf_peak_compute(int32_t kind, int32_t reps, double *tflops);

/* Random row gather: a source of `src_bytes` bytes holds rows of
 * `row_bytes` bytes (a multiple of 16, at most 1024, and src_bytes >=
 * row_bytes); `n_rows` rows picked by a fixed hash of the gather index are
 * read whole and summed.  *gbs = n_rows * row_bytes / time, in GB/s. */
int bpmf_peak_gather(int64_t src_bytes, int32_t row_bytes, int64_t n_rows, int32_t reps, double *gbs);

#ifdef __cplusplus
}
#endif

#endif
