/*
 * selscan_micro.h -- measurement kernels of the MI355X library: achievable
 * rates of the resources the EHH walks use (HBM, int32 VALU, LDS atomics, and
 * a cell-update proxy of the bitmask refinement), measured on the caller's
 * device and stream.  They state the walk's roofline against measured peaks;
 * they compute nothing of the scans.
 *
 * Conventions as in selscan_hip.h: device pointers, caller-owned buffers,
 * `stream` an opaque hipStream_t (NULL = default).  Each call makes one
 * warm-up launch, then `reps` (>= 1) timed launches, waits for them, and
 * returns the mean milliseconds per launch in *ms.
 * Errors: SS_EARG for null or misaligned pointers or bad sizes, SS_EDEV for
 * HIP errors.
 */
#ifndef SELSCAN_MICRO_H
#define SELSCAN_MICRO_H

#include <stddef.h>
#include <stdint.h>

#include "selscan_hip.h"

#ifdef __cplusplus
extern "C" {
#endif

/* uint32 words that d_out of the calls below must hold (64 per CU). */
int ss_micro_out_words(void);

/* HBM stream copy of `bytes` (a multiple of 16; both pointers 16-byte
 * aligned) from d_src to d_dst: 2 * bytes of traffic per launch. */
int ss_micro_copy(const void *d_src, void *d_dst, size_t bytes, int reps, void *stream, double *ms);

/* int32 VALU rate: `iters` iterations of 8 independent add/xor chains per
 * lane in 16 waves per SIMD; *lane_ops = int32 lane-operations per launch. */
int ss_micro_valu(uint32_t *d_out, int iters, int reps, void *stream, double *ms, double *lane_ops);

/* LDS atomic rate: `iters` ds_add_u32 per lane on lane-distinct addresses;
 * *ops = atomics per launch. */
int ss_micro_lds_atomic(uint32_t *d_out, int iters, int reps, void *stream, double *ms, double *ops);

/* Cell-update proxy: every lane holds a 4-word class mask and refines it by
 * `steps` consecutive marker rows of d_rows ([n_rows][4] uint64, read
 * cyclically): AND with the row and its complement, population counts, the
 * larger child kept, C(n,2) of both children summed.  *cells = haplotype-cells
 * refined per launch (64 x 4 bits per lane and row). */
int ss_micro_cell(const uint64_t *d_rows, int64_t n_rows, uint32_t *d_out, int steps, int reps,
                  void *stream, double *ms, double *cells);

#ifdef __cplusplus
}
#endif

#endif /* SELSCAN_MICRO_H */
