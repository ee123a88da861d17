/*
 * corr_peaks.h -- on-device peak probes of libcorr (measurement helpers, not
 * part of the method).
 *
 * The roofline fractions that the library's benchmark reports are taken
 * against the vendor's published MI355X figures and, beside them, against
 * what these probes measure on the device at hand: LDS read bandwidth, dense
 * FP16 MFMA throughput, FP32 and FP64 vector FMA throughput, HBM read
 * bandwidth and the issue rate of the FP32 median instruction. Each probe is
 * one kernel launch on `stream` with a fixed amount of work and no
 * data-dependent addressing; the caller times it (HIP events on the same
 * stream) and divides the work stated below by the time.
 *
 * Conventions: `out` is caller-owned device memory of at least
 * n_blocks * 256 elements of the stated type (one word per thread, written
 * so the compiler keeps the work; the values have no meaning). Returns
 * CORR_OK, CORR_EINVAL for n_blocks < 1, iters < 1, a null pointer or a
 * misaligned buffer, CORR_EHIP for a failed launch. Nothing is allocated.
 */
#ifndef CORR_PEAKS_H
#define CORR_PEAKS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* LDS reads: every thread of n_blocks 256-thread workgroups reads
 * iters * 8 16-byte words (ds_read_b128, a wave's 64 lanes on 1 KiB of
 * consecutive words: no bank conflicts) from a 64 KiB workgroup buffer.
 * Work: n_blocks * 256 * iters * 128 bytes. out: uint32. */
int corr_peak_lds(int n_blocks, int iters, unsigned int* out, void* stream);

/* Dense FP16 matrix cores: every wave of n_blocks 256-thread workgroups issues
 * iters * 4 v_mfma_f32_32x32x16_f16 (four independent accumulators).
 * random_operands = 0: small repeated operand values (the unit's best case);
 * 1: pseudo-random full-mantissa values in (-1, 1), like standardised
 * ensemble data -- the matrix cores draw more power on such data and the
 * clock drops, so this is the ceiling that applies to the correlation
 * contraction. Work: n_blocks * 4 * iters * 4 * 32768 flops. out: float. */
int corr_peak_mfma_f16(int n_blocks, int iters, int random_operands, float* out, void* stream);

/* FP32 vector FMA (unpacked: the library is built without packed FP32):
 * every thread runs 16 independent chains of iters fmaf.
 * Work: n_blocks * 256 * iters * 16 * 2 flops. out: float. */
int corr_peak_valu_f32(int n_blocks, int iters, float* out, void* stream);

/* FP32 three-input median (v_med3_f32, the instruction of the KSG
 * k-nearest-neighbour insertion network): every thread runs 16 independent
 * chains of iters med3. Work: n_blocks * 256 * iters * 16 lane-ops. out: float. */
int corr_peak_valu_med3(int n_blocks, int iters, float* out, void* stream);

/* FP64 vector FMA: every thread runs 8 independent chains of iters fma.
 * Work: n_blocks * 256 * iters * 8 * 2 flops. out: double. */
int corr_peak_valu_f64(int n_blocks, int iters, double* out, void* stream);

/* HBM read stream: n_blocks 256-thread workgroups read the `bytes` bytes at
 * `buf` (device memory, 16-byte aligned, bytes a multiple of 16) once, in
 * 16-byte words, grid-strided. Work: bytes read. out: uint32. */
int corr_peak_hbm_read(const void* buf, size_t bytes, int n_blocks, unsigned int* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CORR_PEAKS_H */
