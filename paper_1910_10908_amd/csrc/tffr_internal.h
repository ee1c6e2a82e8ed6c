// Internal types shared by the host plan (tffr_host.hip) and the kernel sources
// (tffr_range.hip, tffr_azimuth.hip, tffr_misc.hip).  Nothing here crosses the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace tffr {

template <typename R>
struct cplx {
  R x, y;
};

struct half2s {  // two IEEE binary16 values (re, im)
  _Float16 x, y;
};

// Scalar geometry and method constants, passed by value to every kernel.
struct Geo {
  int32_t n_pulses, n_freq, mx, my;
  int32_t nfx, nfy, lognfx, lognfy;  // fine grid sizes (powers of two)
  int32_t W;                         // gridding kernel width (taps)
  int32_t literal;                   // range gridding with the window's lattice transform (Algorithm 1)
  int32_t lit_taps;                  // its taps per sample: 2 q
  int32_t weighting, thresh_mode, band_r, band_b;
  int32_t use_poly, nseg, deg;  // tFFR weight polynomial (float path)
  int32_t sub;                  // range gridding: samples per thread per sub-pass group
  int32_t part_len;             // range gridding: samples per part (part span < fine row)
  int32_t range_mode;           // range gridding: 0 sub-passes, 1 runs of read-add-writes (W <= kRunWindow)
  int32_t yemax;                // azimuth gridding: most (slice, tap) pairs reaching one cell
  int32_t keep0;                // threshold decision for a sample exactly on the lattice
  int32_t run_pair;             // run range kernel takes its samples two at a time (samples < 1/2 cell apart)
  int32_t run_parts;            // run range kernel: parts gridded at once, one LDS row each (1 or 2)
  double beta;                  // ES kernel shape
  double tx_scale;              // kx -> cycles per range pixel: fov_x / (2 pi mx)
  double fov_x;                 // kx -> lattice coordinate: kx * fov_x / (2 pi)
  double fov_y;                 // azimuth scene extent (pixel coordinates Y)
  double a, q, tau;
  double ema2, epa2;  // exp(-a/2), exp(+a/2)
  double inv_g0;      // 1/g(0) for a sample exactly on the lattice
  double near_rel;    // polynomial weights this close to the threshold are re-decided in FP64
  float thr_f;        // float threshold on 1/g: tau (literal) or 1/tau (correlation)
  float near_f;       // near_rel as float
};

// Small device tables owned by the plan, in the compute type R.
template <typename R>
struct Tab {
  const double* k;        // [n_freq]   fast-time wavenumbers
  const double* ku;       // [n_pulses] azimuth wavenumbers (= ky of the slice)
  const double* kx;       // [n_pulses][n_freq] explicit range wavenumbers, or null: Stolt map of k, ku
  const R* ky;            // [n_pulses] ky = ku in the compute type (row phase)
  const int32_t* ystart;  // [n_pulses] first azimuth fine cell of the slice's taps
  const R* ytap;          // [n_pulses][W] azimuth kernel taps of the slice
  const R* deapx;         // [mx] 1 / kernel transform, range
  const R* deapy;         // [my] 1 / kernel transform, azimuth
  const cplx<R>* twx;     // [nfx/64 + 64] two-level table of exp(+2 pi i m / nfx)
  const cplx<R>* twy;     // [nfy/64 + 64] two-level table of exp(+2 pi i m / nfy)
  const R* deapf;         // [n_pulses] 1 / kernel transform at the front end's bins n - n_pulses/2 (grid fgrid)
  const int32_t* ycell_n;  // [nfy][yemax] slices whose taps reach each azimuth cell (padded with 0)
  const R* ycell_w;        // [nfy][yemax] the matching kernel taps (padded with 0)
  const float* poly;      // [kPolyDeg+1][kPolySeg] tFFR weight polynomial (float path), or null
};

enum SampleType { ST_C64 = 0, ST_C128 = 1, ST_H2 = 2 };

// Entropy-step input of the range adjoint: with h12 non-null (the two gradient fields
// interleaved, [n_pulses][mx][2] = (h1, h2)) its range-spectra cotangent is
// alpha h1 + (beta + alpha cblk[column / cb]) h2, where alpha, beta come from the global
// entropy sums: reduced by every block from nparts partial pairs (then block 0 writes
// *loss), or read from stats = {S, E}.
template <typename R>
struct EntComb {
  const cplx<R>* h12;
  const R* cblk;
  int cb;
  const double* partials;
  int nparts;
  const double* stats;
  double* loss;
};

// Launchers (tffr_range.hip, tffr_azimuth.hip, tffr_entstep.hip, tffr_coord.hip, tffr_ffr.hip,
// tffr_misc.hip).  All enqueue on `st` and return the launch status.
template <typename R>
hipError_t launch_fwd_rows(const Geo& g, const Tab<R>& t, int stype, const void* samples,
                           const R* phase, const R* dalong, const R* w, cplx<R>* out,
                           int stage, hipStream_t st);
template <typename R>
hipError_t launch_fwd_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* hx,
                           cplx<R>* img, double* partials, hipStream_t st);
template <typename R>
hipError_t launch_adj_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* cot,
                           cplx<R>* hx, const double* stats, const double* partials, int nparts,
                           double* loss, hipStream_t st);
hipError_t launch_entropy_stats(const double* partials, int nparts, double* stats, double* loss, hipStream_t st);
template <typename R>
hipError_t launch_ent_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* hx, cplx<R>* img,
                           double* partials, R* cblk, cplx<R>* h12, hipStream_t st);
template <typename R>
hipError_t launch_adj_rows(const Geo& g, const Tab<R>& t, int stype, const cplx<R>* hx,
                           const void* samples, const R* phase, const R* dalong, const R* w,
                           cplx<R>* grad_s, R* grad_phase, R* grad_dalong, const EntComb<R>& ec,
                           hipStream_t st);
template <typename R>
hipError_t launch_coord_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* cot, cplx<R>* h0, cplx<R>* h1,
                             hipStream_t st);
template <typename R>
hipError_t launch_coord_grad(const Geo& g, const Tab<R>& t, int cb, int stype, const cplx<R>* cot,
                             const void* samples, const R* phase, const R* dalong, const R* w, cplx<R>* h0,
                             cplx<R>* h1, R* grad_kx, R* grad_ky, hipStream_t st);
template <typename R>
hipError_t launch_row_phase_grad(const Geo& g, const Tab<R>& t, int stype, const void* samples,
                                 const cplx<R>* grad_s, R* grad_phase, R* grad_dalong, hipStream_t st);
template <typename R>
hipError_t launch_weights(const Geo& g, const Tab<R>& t, R* w, unsigned long long* kept_partial,
                          int nblocks, hipStream_t st);
hipError_t launch_sum_u64(const unsigned long long* parts, int n, long long* out, hipStream_t st);
template <typename R>
hipError_t launch_ffr(const Geo& g, const Tab<R>& t, int route, int lmax, int nwg, double* scratch, R* dband,
                      int* status, hipStream_t st);
size_t ffr_scratch_bytes(const Geo& g, int route, int lmax, int nwg);  // scratch of launch_ffr
template <typename R>
hipError_t launch_entropy(const Geo& g, const cplx<R>* img, double* partials, int nparts,
                          double* loss, cplx<R>* grad, hipStream_t st);
template <typename R>
hipError_t launch_rma_front(const Geo& g, const Tab<R>& t, int logj, const cplx<R>* echoes, double xc, int stype,
                            void* out, hipStream_t st);  // tffr_rma.hip
template <typename R>
hipError_t launch_rma_range_fft(int logp, int n_rows, const cplx<R>* pulses, const cplx<R>* ref, cplx<R>* echoes,
                                hipStream_t st);
template <typename R>
hipError_t launch_rma_front_pos(const Geo& g, const Tab<R>& t, int logg, const cplx<R>* echoes, const double* pos,
                                int J, int S, double xc, int stype, void* out, hipStream_t st);
template <typename R>
hipError_t launch_stolt_rows(const Geo& g, const Tab<R>& t, int stype, const void* samples, const R* phase,
                             const R* dalong, int part, cplx<R>* out, hipStream_t st);
template <typename R>
hipError_t launch_fft(int log2n, int batch, int sign, int max_radix, const cplx<R>* in, cplx<R>* out,
                      const cplx<R>* tw, hipStream_t st);

size_t max_dynamic_lds();  // bytes of LDS one workgroup may use on this device
int rows_threads(int logn);  // threads per workgroup of the range-stage kernels for a 2^logn fine row
constexpr int kPolySeg = 32;  // segments of the tFFR weight polynomial on (0, 1)
constexpr int kPolyDeg = 7;   // degree per segment
constexpr int kRunWindow = 8;    // widest kernel of the run range kernel (its pad and halos are 2 kRunWindow cells)
constexpr int kRunHaloInts = 16;  // LDS ints for the run kernel's per-wave halo start cells (up to 16 waves)

}  // namespace tffr
