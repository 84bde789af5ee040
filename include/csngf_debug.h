/*
 * csngf_debug.h - diagnosis, parity and measurement entry points of libcsngf.
 *
 * These calls expose intermediate stages of the hot path so that tests can compare each
 * stage with an independent reference, and give per-kernel device timings for the
 * roofline report.  They use the conventions and error codes of csngf.h.
 */
#ifndef CSNGF_DEBUG_H
#define CSNGF_DEBUG_H

#include <stdint.h>

#include "csngf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Batched complex FFT of length L along a contiguous axis with the library's LDS engine
 * (the transform inside every pencil pass).  in/out: DEVICE pointers to interleaved
 * complex64 [batch][L] (may alias).  inverse = 0: forward, exp(-2 pi i jk/L); 1: inverse,
 * unnormalised.  stream: hipStream_t or NULL (default stream).  Asynchronous on the stream.
 * CSNGF_E_UNSUPPORTED when csngf_supported_length(L) is 0. */
int csngf_debug_fft(const void* in, void* out, int32_t L, int32_t batch, int32_t inverse,
                    void* stream);

/* Run the fused field stage (the first pass of every evaluation, and of the fixed-side
 * precompute) on one volume and return its real outputs: prod6 = the 6 products
 * M n_x^2, M n_y^2, M n_z^2, M n_x n_y, M n_x n_z, M n_y n_z (each [nz][ny][nx] float32,
 * unweighted), and mask = the eroded mask M (uint8 [nz][ny][nx]).
 * R9 != NULL: moving side, vol resampled under R9 (quantised as in csngf_evaluate).
 * R9 == NULL: fixed side, vol used directly (vmask optional).  Px: the x FFT size
 * (0 = smallest supported >= 2 nx - 1).  flags: CSNGF_DEVICE_PTRS for device pointers
 * (vol, vmask, prod6, mask); host otherwise (then synchronous).  With CSNGF_UNSQUARED only
 * the first 3 planes of prod6 are written: M n_x, M n_y, M n_z. */
int csngf_debug_fields(const float* vol, const uint8_t* vmask, csngf_dims d, const double* R9,
                       float eps, int32_t Px, float* prod6, uint8_t* mask, uint32_t flags);

typedef struct {
  char name[32];       /* kernel family */
  int64_t launches;    /* launches timed since the last reset */
  double total_ms;     /* summed device time between HIP events around each launch */
} csngf_kernel_stat;

/* enable != 0: record a HIP event pair on the context's stream around every launch. */
int csngf_profile_enable(csngf_ctx* ctx, int32_t enable);

/* Synchronise the context's stream, fold finished event pairs into per-family totals and
 * copy up to max entries into out; *count receives the number of families. */
int csngf_profile_read(csngf_ctx* ctx, csngf_kernel_stat* out, int32_t max, int32_t* count);

/* Clear the per-family totals and the kept-row counts. */
int csngf_profile_reset(csngf_ctx* ctx);

/* Displacement rows kept by the minimum-overlap pruning (Sec. 3.2), summed over the rotations
 * evaluated while profiling was enabled since the last reset: *z_rows = z-rows with a flag
 * set (of W_z per rotation), *rows = (z, y) rows with a flag set (of W_z W_y), *rotations =
 * the rotations counted.  They are the rows that the pruned inverse passes write and read,
 * so a benchmark can charge those passes the bytes they move.  Any output may be NULL;
 * synchronises the context's streams. */
int csngf_profile_rows(csngf_ctx* ctx, int64_t* z_rows, int64_t* rows, int64_t* rotations);

#ifdef __cplusplus
}
#endif

#endif /* CSNGF_DEBUG_H */
