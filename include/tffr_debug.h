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
 * sign = +1 or -1, no scaling.  max_radix 8 or 16: the Stockham stages' radix (the
 * dense-slice range kernel uses 16, every other kernel 8).  in/out: device complex
 * (dtype TFFR_C64 or TFFR_C128), [batch][n]; in-place allowed.  Synchronises. */
tffr_status tffr_debug_fft(int32_t log2n, int32_t batch, int32_t sign, int32_t max_radix, int32_t dtype,
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

/* Launch configuration the plan chose: range_mode 0 (sub-pass gridding: kernels wider
 * than 8 cells, literal lattice taps), 1 (runs of read-add-writes: every other plan), 2
 * (the same runs two samples at a time: complex64, width 7, rows of 4096 cells and more,
 * samples under half a cell apart) or 3 (the same runs, two parts of a slice at once on
 * twice the threads, each into its own LDS row: slices of several parts on rows of at
 * most 4096 cells);
 * az_cols range columns per azimuth workgroup;
 * ent_fused 1 when tffr_entropy_step uses the fused azimuth kernel.  Any pointer may be
 * NULL. */
tffr_status tffr_debug_plan_config(const tffr_plan *plan, int32_t *range_mode, int32_t *az_cols,
                                   int32_t *ent_fused);

/* Plain-FFR solve route of a TFFR_W_FFR plan: route 0 when every slice has no more samples
 * than lattice points (selected inversion of the frame product), 1 when every slice has
 * more (selected inversion of Sa Sb, the factors' Gram matrices); lattice_max the most
 * lattice points of a slice (plus a margin of 2); solve_status the outcome of the
 * plan-time solve: 0 ok, 1 a vanishing block pivot, 3 an inverse beyond 1e15 of the
 * matrix scale, 2 a slice reaching more lattice points than provided for.  Plan creation
 * fails on a nonzero status unless the environment sets TFFR_FFR_KEEP_SINGULAR=1 (then
 * the plan is kept for inspection and its weights are zero on the failed slices).  Any
 * pointer may be NULL.  TFFR_ERR_ARG for other weightings. */
tffr_status tffr_debug_ffr_route(const tffr_plan *plan, int32_t *route, int32_t *lattice_max,
                                 int32_t *solve_status);

/* Azimuth stage of the fused entropy step alone (the launch inside tffr_entropy_step):
 *   d_hx     [n_pulses][mx] range spectra, read only
 *   d_image  [mx][my] written (as tffr_debug_cols)
 *   d_h12    [n_pulses][mx][2] complex written: (h1, h2) interleaved, h1 the adjoint
 *            azimuth transform of I (ln|I|^2 - c_b) with c_b = ln of column block b's mean
 *            |I|^2, h2 that of I
 *   d_work   workspace of the plan (receives the entropy partial sums and the c_b)
 * TFFR_ERR_UNSUPPORTED when the plan's entropy step does not use the fused kernel. */
tffr_status tffr_debug_ent_cols(tffr_plan *plan, const void *d_hx, void *d_image, void *d_h12,
                                void *d_work, tffr_stream stream);

/* Range adjoint of the fused entropy step alone (the last launch inside
 * tffr_entropy_step), on the gradient fields, entropy partial sums and centring constants
 * that the last tffr_entropy_step or tffr_debug_ent_cols call left in d_work; outputs as
 * tffr_entropy_step (d_loss receives E).  Reads the workspace only, so repeated calls
 * give the same result.  TFFR_ERR_UNSUPPORTED when the plan's entropy step is not fused. */
tffr_status tffr_debug_ent_adj_rows(tffr_plan *plan, const void *d_samples, const void *d_phase,
                                    const void *d_dalong, const void *d_user_w, double *d_loss,
                                    void *d_grad_samples, void *d_grad_phase, void *d_grad_dalong,
                                    void *d_work, tffr_stream stream);

/* Per-launch times of the entropy step: runs tffr_entropy_step `nsteps` times (arguments
 * as there) with a HIP event recorded on `stream` before each of its launches and after
 * the last, synchronising after every step, and returns the average time between
 * consecutive events, i.e. of each launch in the step's own order and data flow:
 *   ms_out  host float[7], receives *nkern averages (ms)
 *   nkern   receives the number of launches (3 to 5)
 *   names   host const char*[7] or NULL, receives the kernels' names (static strings)
 * The events are created and destroyed inside the call. */
tffr_status tffr_debug_step_kernel_times(tffr_plan *plan, const void *d_samples, const void *d_phase,
                                         const void *d_dalong, const void *d_user_w, void *d_image, double *d_loss,
                                         void *d_grad_samples, void *d_grad_phase, void *d_grad_dalong, void *d_work,
                                         tffr_stream stream, int32_t nsteps, float *ms_out, int32_t *nkern,
                                         const char **names);

/* Marginal per-launch times of the entropy step, without events between its launches:
 * times `nsteps` plain steps (HIP events on `stream` around the loop only), then, for each
 * launch i of the step, `nsteps` steps in which launch i is issued twice back to back;
 * ms_out[i] is the difference of the two per-step averages, i.e. what one more launch i
 * adds to the step in its steady state.  Every launch of the step overwrites its outputs
 * (none accumulates), so repeating one leaves them as in a plain step; one plain step
 * runs last, and the outputs are those of one step when the call returns.  Arguments
 * and outputs as for tffr_debug_step_kernel_times; the call synchronises `stream`. */
tffr_status tffr_debug_step_kernel_marginal_times(tffr_plan *plan, const void *d_samples, const void *d_phase,
                                                  const void *d_dalong, const void *d_user_w, void *d_image,
                                                  double *d_loss, void *d_grad_samples, void *d_grad_phase,
                                                  void *d_grad_dalong, void *d_work, tffr_stream stream,
                                                  int32_t nsteps, float *ms_out, int32_t *nkern, const char **names);

#ifdef __cplusplus
}
#endif

#endif /* TFFR_DEBUG_H */
