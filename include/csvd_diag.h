/*
 * csvd_diag.h -- measurement probes of the MI355X solver library.
 *
 * Not part of the method: these calls measure the memory system so that the
 * kernels of the library can be reported against what the hardware delivers
 * for their access pattern, next to the published peaks.
 */
#ifndef CSVD_DIAG_H
#define CSVD_DIAG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Random-row gather ceiling of the sparse products of the block step (the
 * operator apply of Algorithm 1, step 1): out_rows output rows, each the sum
 * of per_out rows of 64 doubles (512 bytes) drawn uniformly at random from a
 * table of table_rows rows (indices from a generator seeded with `seed`,
 * sorted within each output row), with no matrix values.  variant 0 uses the
 * lane layout of the library's block products (lane c of the 16 lanes of a
 * row reads columns 4c..4c+3); variant 1 lets each load instruction cover a
 * contiguous half row.  Allocates its own table, indices and output on the
 * current device (freed before return), runs two warm-up launches and then
 * `reps` timed launches on the default stream.
 * Output: *ms_per_launch, the average duration of one launch in ms.
 * Errors: CSVD_EINVAL (sizes, variant), CSVD_ENOMEM, CSVD_EDEVICE. */
int csvd_probe_gather(int64_t table_rows, int32_t variant, int64_t out_rows, int32_t per_out, uint64_t seed,
                      int32_t reps, double *ms_per_launch);

#ifdef __cplusplus
}
#endif

#endif /* CSVD_DIAG_H */
