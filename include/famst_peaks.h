/* Measured ceilings of one MI355X (gfx950) for the rooflines of the
 * screening kernels: matrix-core throughput of the three MFMA forms the
 * screening issues, and HBM copy / read bandwidth.  Measurement helpers
 * beside libfamst, not part of the method; built into libfamst_peaks.so.
 *
 * Conventions as in famst.h: int status (0 = ok, negative = error), device
 * pointers unless marked host, work enqueued on the given hipStream_t (NULL:
 * the null stream).  Every call synchronises its stream before returning
 * its host outputs and allocates nothing. */
#ifndef FAMST_PEAKS_H
#define FAMST_PEAKS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Matrix-core throughput.  precision: 0 = v_mfma_f32_16x16x4_f32,
 * 1 = v_mfma_f32_16x16x32_bf16, 2 = v_mfma_scale_f32_16x16x128_f8f6f4 (e4m3
 * operands, unit scales).  Every wave of a full-chip grid (two blocks of four
 * waves per CU) issues `iters` rounds of eight independent MFMAs on register
 * operands; the result is dense flops / elapsed time.
 *   sink   : device, 4 bytes, written only in a case that cannot occur (it
 *            keeps the products live); caller-owned.
 *   tflops : host, out.
 * Errors: -1 (FAMST_EINVAL) for an unknown precision or iters < 1, -5
 * (FAMST_EHIP) for a HIP error. */
int famst_peak_mfma(int32_t precision, int32_t iters, float* sink, double* tflops, void* stream);

/* HBM bandwidth over `bytes` (a multiple of 16) of caller-owned device
 * memory: `reps` copies src -> dst (bytes read + bytes written per copy)
 * and `reps` reads of src (a sum that lands in `sink` only in a case that
 * cannot occur).
 *   src, dst : device, `bytes` each, 16-byte aligned; dst is overwritten.
 *   sink     : device, 4 bytes.
 *   copy_gbps, read_gbps : host, out (1e9 bytes per second).
 * Errors: -1 for bytes not a positive multiple of 16, misaligned or null
 * pointers, reps < 1; -5 for a HIP error. */
int famst_peak_hbm(const void* src, void* dst, size_t bytes, int32_t reps, float* sink,
                   double* copy_gbps, double* read_gbps, void* stream);

#ifdef __cplusplus
}
#endif
#endif
