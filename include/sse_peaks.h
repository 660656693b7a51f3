/* sse_peaks.h -- C ABI of libsse_peaks.so: throughput microbenchmarks of the
 * GPU units the scatter simulation is bound by.
 *
 * The simulation is neither a dense contraction nor HBM-streaming work: its
 * transport runs on the vector ALUs (binary32 and 32-bit integer arithmetic,
 * the Philox generator's 32 x 32 -> 64-bit multiplies, selects), gathers the
 * attenuation map, emission sampler and LUT at random through the caches, and
 * accumulates its sinogram with random atomic adds.  The roofline of such a
 * kernel needs the measured peak of each of these on the device it runs on;
 * this library measures them.  It is measurement support, separate from the
 * scatter-estimation library, and allocates its own temporary buffers.
 */
#ifndef SSE_PEAKS_H
#define SSE_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Measured rates on one device (per second unless stated).  VALU rates are
 * lane-operations (one wave64 instruction = 64 lane-operations), from loops
 * of 8 independent chains of one instruction each:
 *   v_add_u32, v_xor_b32, v_fma_f32, v_mad_u64_u32 (the 32 x 32 -> 64-bit
 *   multiply-add), v_cndmask_b32 (a select, with its compare), v_log_f32 (a
 *   transcendental).
 * Gathers: random independent 4-byte loads over buffers of 2 MiB (held in
 * one XCD's L2), 32 MiB (beyond L2, inside the last-level cache) and 2 GiB
 * (HBM); one load per lane, counted per lane.  Atomics: random 4-byte
 * integer and 8-byte binary64 adds without return over a buffer of
 * atomic_bins entries.  copy_bytes_per_s: a plain device-to-device copy
 * kernel (bytes read + written).  sclk_mhz: the shader clock during the VALU
 * loops (s_memtime against the 100 MHz s_memrealtime). */
typedef struct {
  double sclk_mhz;
  double valu_add, valu_xor, valu_fma, valu_mad64, valu_cndmask, valu_log;
  double gather_l2, gather_llc, gather_hbm;
  double atomic_u32, atomic_f64;
  double copy_bytes_per_s;
  uint64_t atomic_bins;
  uint64_t cus;            /* compute units of the device */
} sse_peaks;

/* Run every microbenchmark on HIP device `device` (synchronous; about a
 * second).  atomic_bins: entries of the atomic-add buffer (0: 206 397 408,
 * the clinical TOF sinogram).  Returns 0, or a negative HIP error code. */
int sse_measure_peaks(int device, uint64_t atomic_bins, sse_peaks* out);

#ifdef __cplusplus
}
#endif
#endif
