/*
 * tffr.h -- C ABI of libtffr: thresholded non-uniform Fourier frame reconstruction
 * (tFFR) of Stolt-mapped stripmap-SAR phase history on one AMD MI355X (gfx950).
 *
 * Method: McKay, Gelb, Jayasuriya, Monga, "Thresholded Non-Uniform Fourier
 * Frame-Based Reconstruction for Stripmap SAR".  Algorithm 1 takes the Fourier data
 * f_hat(lambda^1_n, lambda^2_p), the uniform grid {l_m} and a threshold tau > 0 and
 * returns the SAR image; this library takes the phase-history samples, the radar
 * wavenumbers that fix their coordinates, the weighting method with its window and
 * threshold parameters, and returns the image (forward), the adjoint of that map
 * (gradients), and an image-entropy loss.
 *
 * Conventions shared by every call:
 *  - Samples are [n_pulses][n_freq], row-major: row n is one azimuth slice (pulse) at
 *    azimuth wavenumber ku[n]; column p is fast-time wavenumber k[p].  Sample (n, p)
 *    sits at kx = sqrt(4 k_p^2 - ku_n^2), ky = ku_n (Stolt map, Sec. II-A).
 *  - Images are [mx][my], row-major and RANGE-MAJOR: element (jx, jy) is at offset
 *    jx*my + jy and is the pixel at X = (jx - mx/2) fov_x/mx (range),
 *    Y = (jy - my/2) fov_y/my (azimuth), both relative to the scene centre.
 *  - The forward map is I[jx,jy] = sum_{n,p} c[n,p] exp(+i (kx X + ky Y)) with
 *    c = D (s * exp(i (phase[n] + ky[n] dalong[n]))) and D the weights of the chosen
 *    method (Eq. (1); Eqs. (3)-(4) and (8) reach it with the window truncated).
 *    It is evaluated by gridding with an exponential-of-semicircle kernel of
 *    kernel_width taps on a grid upsampfac times finer, inverse FFT, and division by
 *    the kernel's transform.  No global normalisation is applied.
 *  - Complex data are interleaved (re, im).  dtype TFFR_C64: float; TFFR_C128: double;
 *    TFFR_C64_FP16IN: samples stored as two IEEE half values, everything else float.
 *    "real" below means float for C64 / C64_FP16IN and double for C128.
 *  - Device pointers are HIP device memory on the current device; the caller owns
 *    every buffer it passes.  The plan owns only small device tables.
 *  - Calls that take a stream only enqueue work on it and never synchronise, except
 *    tffr_kept_count.  A plan is immutable after creation; concurrent calls on one
 *    plan need separate workspaces.
 *  - Every call returns a tffr_status; nothing throws or aborts across the ABI.
 *    Argument and geometry errors are detected on the host before any launch.
 */
#ifndef TFFR_H
#define TFFR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tffr_plan tffr_plan;
typedef void *tffr_stream; /* a hipStream_t; NULL is the null stream */

typedef enum {
  TFFR_OK = 0,
  TFFR_ERR_ARG = 1,          /* bad size, pointer or parameter value               */
  TFFR_ERR_EVANESCENT = 2,   /* some sample has 4 k^2 <= ku^2                       */
  TFFR_ERR_NONMONOTONE = 3,  /* k (or kx along a slice) is not strictly increasing  */
  TFFR_ERR_LAYOUT = 4,       /* buffer misaligned, or ky not constant along a slice  */
  TFFR_ERR_UNSUPPORTED = 5,  /* width, dtype, grid size or FFR band not supported   */
  TFFR_ERR_SINGULAR = 6,     /* plain-FFR solve numerically singular in FP64        */
  TFFR_ERR_NOMEM = 7,        /* device or host allocation of plan tables failed     */
  TFFR_ERR_HIP = 8,          /* a HIP runtime call failed                           */
  TFFR_ERR_SCRATCH = 9       /* tffr_entropy_step_noalloc: the plan's step needs more
                                than TFFR_SCRATCH_BYTES                               */
} tffr_status;

/* Size of the static device array tffr_entropy_step_noalloc works in (per GPU). */
#define TFFR_SCRATCH_BYTES (32u << 20)

/* Weighting methods: the alpha_n / D of Eqs. (1), (4) and (8). */
enum {
  TFFR_W_NONE = 0, /* D = I                                                          */
  TFFR_W_QUAD = 1, /* trapezoid quadrature in lambda along each slice (Sec. II-B)     */
  TFFR_W_FFR = 2,  /* plain FFR: D = B_r(pinv(Psi W)) per slice (Eq. (8))              */
  TFFR_W_TFFR = 3, /* tFFR: D = R_tau(pinv(diag(Psi W))) (Sec. III-B, III-C)           */
  TFFR_W_USER = 4  /* caller-supplied diagonal weights                                */
};

/* What R_tau compares (Sec. III-B): the entries of the inverted diagonal as written
 * (keep iff |1/g| >= tau), or the correlation g itself (keep iff g >= tau).  The FP32
 * and FP64 paths take the same decision (values within 1e-5 of tau are decided in FP64). */
enum { TFFR_THRESH_LITERAL = 0, TFFR_THRESH_CORRELATION = 1 };

enum { TFFR_C64 = 0, TFFR_C128 = 1, TFFR_C64_FP16IN = 2 };

/* Range gridding.  TFFR_GRID_ES: exponential-of-semicircle kernel on a grid upsampfac
 * times finer than the image, deapodised by the kernel's transform; approximates the
 * weighted sum of Eq. (1) to ~1e-6 at width 7.  TFFR_GRID_LITERAL: Algorithm 1 / Eq. (8)
 * as printed: the window's own transform R_W(l_m - lambda) at the 2q lattice points
 * |l_m - lambda| < q of the image lattice itself (no oversampling), inverse FFT, division
 * by w(x) = exp(-a |x - 1/2|); the truncation error of the paper's method is kept.  The
 * azimuth stage is the same in both. */
enum { TFFR_GRID_ES = 0, TFFR_GRID_LITERAL = 1 };

typedef struct {
  int32_t n_pulses;     /* slices n (azimuth), >= 1                                   */
  int32_t n_freq;       /* samples p per slice (fast-time frequency), >= 1            */
  int32_t mx, my;       /* image size (range, azimuth), even, 2..16384               */
  double fov_x, fov_y;  /* scene extents in metres, > 0                               */
  int32_t weighting;    /* TFFR_W_*                                                   */
  double window_a;      /* w(x) = exp(-a |x - 1/2|), a = 0.01 in Sec. IV; >= 0        */
  double q;             /* truncation of W and Psi in lattice units, >= 1 (default 3) */
  int32_t band_r;       /* plain-FFR band B_r, r = 2 in Sec. IV; 0..8 (the solve covers
                           max(r, half-band of the frame product) diagonals)           */
  double tau;           /* threshold, tau = 0.97 in Sec. IV; > 0                      */
  int32_t thresh_mode;  /* TFFR_THRESH_*                                              */
  int32_t kernel_width; /* gridding taps: 2..16 (7 gives ~1e-6 relative error)        */
  double upsampfac;     /* fine grid >= upsampfac * image size, rounded up to 2^k; 1.25..4 */
  int32_t dtype;        /* TFFR_C64, TFFR_C128, TFFR_C64_FP16IN                        */
  int32_t gridding;     /* TFFR_GRID_ES (default) or TFFR_GRID_LITERAL (integer q <= 8,
                           mx a power of two >= 64)                                    */
} tffr_params;

/* Paper defaults: a = 0.01, tau = 0.97, r = 2 (Sec. IV, Baselines); q = 3, tFFR with
 * the literal threshold, width 7, upsampfac 2, complex64.  Sizes are set to 0. */
void tffr_default_params(tffr_params *p);

/* Host-only check of params and geometry; no HIP call.  k: host [n_freq] rad/m,
 * ku: host [n_pulses] rad/m.  Returns the status tffr_plan_create would return for
 * these arguments before touching the device. */
tffr_status tffr_validate(const tffr_params *p, const double *k, const double *ku);

/* Create a plan on the current HIP device.  k and ku are copied.  Builds the device
 * tables (kernel deapodisation, twiddles, per-slice azimuth taps, tFFR weight
 * polynomial).  For TFFR_W_FFR it also solves the plain-FFR weights of every slice on
 * the device and keeps them (Eq. (8)): by selected inversion of the banded frame product
 * when no slice has more samples than lattice points (and the band, widened to r, is at
 * most 8), or, when every slice has more samples than lattice points (the product has
 * rank L < P), of the product of the factors' Gram matrices, pinv(A B^T) = B (B^T B)^-1
 * (A^T A)^-1 A^T (q <= 3, r times the widest sample spacing plus 2q at most 10); any
 * other geometry gives TFFR_ERR_UNSUPPORTED, and a slice whose matrix is numerically
 * singular in FP64 (a vanishing block pivot, or an inverse of 1e15 or more over the
 * matrix scale after diagonal equilibration) gives TFFR_ERR_SINGULAR.  Synchronises the
 * device.  *out is NULL on error. */
tffr_status tffr_plan_create(const tffr_params *p, const double *k, const double *ku,
                             tffr_plan **out);

/* Plans from explicit sample coordinates instead of the Stolt map: any geometry with
 * the slice structure the method relies on (Sec. II-A: each slice has one ky, its
 * samples are non-uniform in kx only; Algorithm 1 loops over such slices).
 *   kx, ky: host [n_pulses][n_freq] rad/m, copied (the plan keeps kx on the device,
 *           8 bytes per sample).  Along every slice n, ky[n][p] must be one value
 *           (else TFFR_ERR_LAYOUT) and kx[n][p] strictly increasing in p (else
 *           TFFR_ERR_NONMONOTONE); non-finite values give TFFR_ERR_ARG.
 * The plan then behaves as one from tffr_plan_create with kx, ky in place of the
 * Stolt map (dalong scales with that ky).  tffr_validate_xy is the host-only check. */
tffr_status tffr_validate_xy(const tffr_params *p, const double *kx, const double *ky);
tffr_status tffr_plan_create_xy(const tffr_params *p, const double *kx, const double *ky,
                                tffr_plan **out);

void tffr_plan_destroy(tffr_plan *plan);

/* Bytes of caller-owned device workspace every forward / adjoint / entropy / weights
 * call needs (three [n_pulses][mx] complex arrays of per-slice range spectra plus
 * reduction scratch).  0 for NULL. */
size_t tffr_workspace_bytes(const tffr_plan *plan);

/* Sizes chosen by the plan: fine grid in range and azimuth, ES kernel shape beta,
 * plain-FFR half-bandwidth of the frame product (0 for other methods). */
tffr_status tffr_plan_info(const tffr_plan *plan, int32_t *nfine_x, int32_t *nfine_y,
                           double *beta, int32_t *ffr_halfband);

/* Materialise the weights of the plan's method into d_w (device, real):
 *   diagonal methods: [n_pulses][n_freq];  TFFR_W_FFR: [n_pulses][n_freq][2r+1] with
 *   entry [n][p][r+o] = D_{p,p+o} of slice n (0 past the row ends).
 * TFFR_W_USER is rejected (TFFR_ERR_ARG).  Enqueued on `stream`. */
tffr_status tffr_weights(tffr_plan *plan, void *d_w, void *d_work, tffr_stream stream);

/* Number c of samples the threshold keeps (Sec. III-C), computed on the device and
 * copied to *count.  Synchronises `stream`.  For non-tFFR methods c = n_pulses*n_freq. */
tffr_status tffr_kept_count(tffr_plan *plan, void *d_work, int64_t *count, tffr_stream stream);

/* Forward (image formation):
 *   d_samples  [n_pulses][n_freq] complex (dtype), read only
 *   d_phase    [n_pulses] real, per-pulse phase error phi in rad, or NULL (zeros)
 *   d_dalong   [n_pulses] real, along-track position error du in m, or NULL (zeros)
 *   d_user_w   NULL to compute the plan's weights on the fly; otherwise weights in the
 *              layout of tffr_weights (required for TFFR_W_USER)
 *   d_image    [mx][my] complex, written (range-major)
 *   d_work     tffr_workspace_bytes() bytes of device scratch */
tffr_status tffr_forward(tffr_plan *plan, const void *d_samples, const void *d_phase,
                         const void *d_dalong, const void *d_user_w, void *d_image,
                         void *d_work, tffr_stream stream);

/* Range-migration front end (Sec. II-A: frequency-domain mapping and matched filter
 * before the Stolt change of variables):
 *   d_echoes    [n_positions][n_freq] complex in the compute type (complex float for
 *               TFFR_C64 and TFFR_C64_FP16IN, complex double for TFFR_C128): raw echoes
 *               at along-track positions u_j = (j - n_positions/2) du, fast-time
 *               wavenumbers k of the plan; read only
 *   d_samples   [n_pulses][n_freq] samples in the plan's sample type, written:
 *               s[n][p] = exp(+i kx[n][p] xc) sum_j e[j][p] exp(-i ku_n u_j)
 * xc is the reference range (m) that the matched filter removes.  The plan must come
 * from tffr_plan_create with ku_n = (n - floor(n_pulses/2)) 2 pi / (n_positions du)
 * (checked to 1e-9 of the bin width, else TFFR_ERR_ARG); n_positions a power of two, at least 64
 * and n_pulses (TFFR_ERR_ARG), at most 16384 (8192 for TFFR_C128; else
 * TFFR_ERR_UNSUPPORTED).  No workspace.  Enqueued on `stream`. */
tffr_status tffr_rma_front_end(tffr_plan *plan, const void *d_echoes, int32_t n_positions, double du,
                               double xc, void *d_samples, tffr_stream stream);

/* Range FFT and matched filter (Sec. II-A: the data are taken to the frequency domain and
 * matched filtered before the azimuth transform):
 *   d_pulses  [n_positions][n_freq] complex (complex128 for TFFR_C128, else complex64):
 *             each pulse's n_freq baseband time samples at the rate of the bandwidth
 *   d_ref     [n_freq] complex reference spectrum of the matched filter, or NULL (ones:
 *             data already dechirped)
 *   d_echoes  [n_positions][n_freq] complex, written (may alias d_pulses):
 *             d_echoes[j][p] = ref[p] sum_t d_pulses[j][t] exp(-2 pi i (p - n_freq/2) t / n_freq),
 *             the centred frequency bins, p <-> k_p ascending, as tffr_rma_front_end takes.
 * n_freq must be a power of two, 64 ... 16384 (8192 for TFFR_C128), else
 * TFFR_ERR_UNSUPPORTED; TFFR_ERR_ARG for NULL buffers or n_positions < 1; enqueue only. */
tffr_status tffr_rma_range_fft(tffr_plan *plan, const void *d_pulses, int32_t n_positions, const void *d_ref,
                               void *d_echoes, tffr_stream stream);

/* The same front end for echoes recorded off their nominal positions (per-pulse
 * along-track position errors): echo j was recorded at u_j + dpos[j], and the azimuth sum
 *   d_samples[n][p] = exp(+i kx(n, p) xc) sum_j d_echoes[j][p] exp(-i ku_n (u_j + dpos[j]))
 * is taken at those true positions (no longer a DFT: a type-1 NUFFT at the positions,
 * ES kernel of the plan's width on a periodic grid of at least 2 n_pulses cells).
 *   dpos  HOST array [n_positions] of position errors in metres, finite; the true
 *         positions must increase strictly with j and stay within one period n_positions du
 *         (else TFFR_ERR_NONMONOTONE).
 * Other arguments and their errors as tffr_rma_front_end.  The positions are copied to a
 * plan-owned device buffer: the call first synchronises `stream` (an earlier call's launch
 * may still read the buffer), then enqueues the transform.  Calls on one plan from
 * different host threads must not overlap. */
tffr_status tffr_rma_front_end_pos(tffr_plan *plan, const void *d_echoes, int32_t n_positions, double du,
                                   const double *dpos, double xc, void *d_samples, tffr_stream stream);

/* Stolt-interpolation baseline image (Sec. II-A; Sec. IV, Baselines): along every slice
 * the (phased) samples are interpolated linearly onto the integer lattice l between the
 * slice's first and last sample (kx = 2 pi l / fov_x; zero outside), and
 *   d_image[jx][jy] = sum_n sum_l S_n(l) exp(+i (2 pi l X_jx / fov_x + ky_n Y_jy))
 * with the pixels of tffr_forward.  The plan's weighting is not used.  Arguments as for
 * tffr_forward (no weights).  mx must be a power of two (TFFR_ERR_UNSUPPORTED). */
tffr_status tffr_stolt_image(tffr_plan *plan, const void *d_samples, const void *d_phase,
                             const void *d_dalong, void *d_image, void *d_work, tffr_stream stream);

/* Adjoint / backward of tffr_forward for a real loss L(I):
 *   d_grad_image   [mx][my] complex, dL/dRe I + i dL/dIm I, read only
 *   d_samples      [n_pulses][n_freq] complex (dtype); needed only when d_grad_phase or
 *                  d_grad_dalong is non-NULL, else may be NULL
 *   d_phase, d_dalong, d_user_w as in tffr_forward
 *   d_grad_samples [n_pulses][n_freq] complex (float for C64/C64_FP16IN), written:
 *                  exp(-i psi_n) D^T A^H grad_image
 *   d_grad_phase   [n_pulses] real or NULL: dL/dphi_n = sum_p Re(conj(g'_np) i s'_np)
 *   d_grad_dalong  [n_pulses] real or NULL: ky_n dL/dphi_n
 * With the gradient outputs NULL this is the plain adjoint operator A'^H. */
tffr_status tffr_adjoint(tffr_plan *plan, const void *d_grad_image, const void *d_samples,
                         const void *d_phase, const void *d_dalong, const void *d_user_w,
                         void *d_grad_samples, void *d_grad_phase, void *d_grad_dalong,
                         void *d_work, tffr_stream stream);

/* Image entropy E = -sum p_j ln p_j, p_j = |I_j|^2 / sum |I|^2, the focus criterion
 * for autofocus-style refinement (the paper's TBED of Eq. (10) uses region entropies):
 *   d_image       [mx][my] complex, read only
 *   d_loss        device double[1], written
 *   d_grad_image  [mx][my] complex or NULL: -(2/S)(ln p_j + E) I_j (0 where I_j = 0) */
tffr_status tffr_entropy(tffr_plan *plan, const void *d_image, double *d_loss,
                         void *d_grad_image, void *d_work, tffr_stream stream);

/* One autofocus-style step, fused: forward image, image entropy E (as tffr_entropy),
 * and the adjoint of dE/dI (as tffr_adjoint with grad_image = tffr_entropy's gradient)
 * without materialising dE/dI.  The gradient is alpha I (ln|I|^2 - c) + (beta + alpha c) I
 * with alpha, beta fixed by the global sums of |I|^2 and |I|^2 ln|I|^2, so one azimuth
 * kernel forms each image column, its share of the sums and the adjoint azimuth
 * transforms of both fields; the range adjoint combines them.  Three kernel launches
 * (four when the image has more than 1024 column blocks).
 *   arguments as in tffr_forward / tffr_adjoint; d_image is written (range-major) and
 *   d_loss (device double[1]) receives E; d_samples is required; d_grad_phase and
 *   d_grad_dalong may be NULL. */
tffr_status tffr_entropy_step(tffr_plan *plan, const void *d_samples, const void *d_phase,
                              const void *d_dalong, const void *d_user_w, void *d_image,
                              double *d_loss, void *d_grad_samples, void *d_grad_phase,
                              void *d_grad_dalong, void *d_work, tffr_stream stream);

/* tffr_entropy_step without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc): it works in a static device array of TFFR_SCRATCH_BYTES (32 MiB) that the
 * library holds on each GPU it runs on until the process ends, and calls no allocating
 * routine.  Arguments and results as tffr_entropy_step, all caller-owned.
 *  - TFFR_ERR_SCRATCH when the plan's step needs more than TFFR_SCRATCH_BYTES (its range
 *    spectra and two gradient fields take 24 n_pulses mx bytes in complex64: up to
 *    512 x 1024 -> 1024^2 and 1024 x 2048 -> 1024^2 fit, 2048 x 4096 -> 2048^2 does not);
 *    TFFR_ERR_HIP when the array's device address could not be resolved at plan creation.
 *  - Every call on one GPU shares that GPU's array and leaves its contents behind; the
 *    step writes every scratch value before reading it, so nothing needs clearing, but
 *    calls that overlap on one GPU (concurrent streams, threads) race and corrupt each
 *    other.  Serialise them. */
tffr_status tffr_entropy_step_noalloc(tffr_plan *plan, const void *d_samples, const void *d_phase,
                                      const void *d_dalong, const void *d_user_w, void *d_image,
                                      double *d_loss, void *d_grad_samples, void *d_grad_phase,
                                      void *d_grad_dalong, tffr_stream stream);

/* Gradients with respect to the sample coordinates, for refining the geometry itself
 * (the method's weights held fixed as constants of the geometry):
 *   d_grad_image  [mx][my] complex G = dL/dRe I + i dL/dIm I, read only
 *   d_samples, d_phase, d_dalong, d_user_w as in tffr_forward (d_samples required)
 *   d_grad_kx     [n_pulses][n_freq] real, written: dL/dkx = Re(i c conj(A^H(X G)))
 *   d_grad_ky     [n_pulses] real, written: dL/dky_n = sum_p Re(i c conj(A^H(Y G)))
 * with c the weighted, phased sample and A^H the adjoint sum; X, Y the pixel coordinates
 * of the image convention (dI/dkx = i X c e^{i(kx X + ky Y)}).  Uses the workspace's two
 * range-spectra arrays.  TFFR_ERR_UNSUPPORTED when two fine rows / columns do not fit in
 * LDS (fine grids of 16384 points). */
tffr_status tffr_coord_grad(tffr_plan *plan, const void *d_grad_image, const void *d_samples,
                            const void *d_phase, const void *d_dalong, const void *d_user_w,
                            void *d_grad_kx, void *d_grad_ky, void *d_work, tffr_stream stream);

/* Per-slice phase and position gradients from a sample cotangent computed elsewhere:
 *   d_samples      [n_pulses][n_freq] complex (dtype), the raw samples s
 *   d_grad_samples [n_pulses][n_freq] complex (real type of the plan): dL/dRe s + i dL/dIm s
 *   d_grad_phase   [n_pulses] real, written: dL/dphi_n = sum_p (Im g_np Re s_np - Re g_np Im s_np)
 *   d_grad_dalong  [n_pulses] real or NULL, written: ky_n dL/dphi_n
 * This is the reduction tffr_adjoint performs when its gradient outputs are non-NULL
 * (the row phase exp(i(phi_n + ky_n du_n)) multiplies every sample of slice n, so
 * dL/dphi_n = sum_p Re(conj(dL/ds') i s') = sum_p Re(conj(g) i s)); FP64 accumulation. */
tffr_status tffr_row_phase_grad(tffr_plan *plan, const void *d_samples, const void *d_grad_samples,
                                void *d_grad_phase, void *d_grad_dalong, tffr_stream stream);

const char *tffr_status_string(tffr_status s);

#ifdef __cplusplus
}
#endif

#endif /* TFFR_H */
