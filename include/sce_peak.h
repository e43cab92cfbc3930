/*
 * sce_peak.h -- throughput probes of the MI355X (gfx950) units the spectral
 * electrostatic kernels are bound by, for the roofline denominators: the
 * published peaks assume the 2.4 GHz peak clock, while the chip runs lower
 * under sustained matrix-core or vector load (power limit).
 *
 * Each probe launches, on the current HIP device and its null stream, a grid
 * of several blocks per compute unit whose waves run independent dependency
 * chains of one instruction kind on register operands (no memory traffic
 * besides one store per thread at the end), times it with HIP events and
 * returns the achieved rate in TFLOP/s (FMA = 2 flops; a 16x16x32 matrix
 * instruction = 16384 flops).  Operands carry varying mantissas.  The
 * sustained rate depends on the operands' values (switching activity sets
 * the power, which sets the clock): the matrix-core probe uses the pattern of
 * the split-precision kernels, an FP16 hi part of magnitude 0.4-0.75 and a lo
 * part of about 1e-3, multiplied as lo*hi, hi*lo, hi*hi into 16 accumulators
 * per wave at 4 waves per SIMD.  ms (may be NULL) receives the timed launch's
 * duration.  Device memory: one small buffer, allocated and freed by each
 * call.
 *
 * Returns 0, or -3 after a HIP error (the message from hipGetErrorString is
 * printed to stderr).
 */
#ifndef SCE_PEAK_H
#define SCE_PEAK_H

#ifdef __cplusplus
extern "C" {
#endif

/* v_mfma_f32_16x16x32_f16: dense FP16 matrix-core rate (FP32 accumulation). */
int sce_peak_mfma_f16(double *tflops, double *ms);

/* v_fma_f32 (one FP32 FMA per lane per instruction; this build never issues
 * packed FP32, so the published figure's packed dual issue is not counted). */
int sce_peak_fma_f32(double *tflops, double *ms);

/* v_fma_f64 (FP64 vector FMA). */
int sce_peak_fma_f64(double *tflops, double *ms);

#ifdef __cplusplus
}
#endif

#endif /* SCE_PEAK_H */
