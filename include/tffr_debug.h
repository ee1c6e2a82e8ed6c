/*
 * tffr_debug.h -- per-pass hooks of libtffr for parity tests of single stages.
 *
 * These run one stage of the forward path in isolation so that a test can compare it
 * with an independent reference of that stage alone.  Same conventions as tffr.h.
 */
#ifndef TFFR_DEBUG_H
#define TFFR_DEBUG_H

#include "tffr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* `batch` in-LDS FFTs of length 2^log2n (6 <= log2n <= 14), the transform used by the
 * 2-D inverse FFT of Algorithm 1: out[b][j] = sum_g in[b][g] exp(sign 2 pi i g j / n),
 * sign = +1 or -1, no scaling.  in/out: device complex (dtype TFFR_C64 or TFFR_C128),
 * [batch][n]; in-place allowed. */
tffr_status tffr_debug_fft(int32_t log2n, int32_t batch, int32_t sign, int32_t dtype,
                           const void *d_in, void *d_out, tffr_stream stream);

/* Range stage of the forward path for every slice.  stage 0: the gridded fine rows
 * [n_pulses][nfine_x] (spread of the weighted, phased samples with the plan's kernel,
 * before any FFT); stage 1: the range-transformed, deapodised rows [n_pulses][mx].
 * Arguments as tffr_forward; d_out is device complex of the plan's compute type. */
tffr_status tffr_debug_rows(tffr_plan *plan, int32_t stage, const void *d_samples,
                            const void *d_phase, const void *d_dalong, const void *d_user_w,
                            void *d_out, tffr_stream stream);

/* Azimuth stage of the forward path alone: d_hx [n_pulses][mx] range spectra (as
 * tffr_debug_rows stage 1 returns them) -> d_image [mx][my].  Same launch as inside
 * tffr_forward. */
tffr_status tffr_debug_cols(tffr_plan *plan, const void *d_hx, void *d_image, tffr_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* TFFR_DEBUG_H */
