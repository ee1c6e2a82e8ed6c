// Host side of libtffr: parameter and geometry validation, plan tables, workspace
// layout and the C ABI entry points declared in include/tffr.h and tffr_debug.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "tffr.h"
#include "tffr_debug.h"
#include "tffr_internal.h"

using tffr::cplx;

namespace {

constexpr double kPi = 3.141592653589793;
constexpr int kMaxLogN = 14;
constexpr int kPartials = 1024;  // reduction blocks for the kept count
constexpr int kEntropyParts = 256;  // reduction blocks for the entropy
constexpr int kFuseStatsMax = 1024;  // entropy step: adjoint blocks reduce up to this many partials
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// ---------------------------------------------------------------- window transforms
// Same closed forms as the device code: centred finite-interval cosine transforms of
// exp(-a|t|) and exp(+a|t|) over [-1/2, 1/2].
double r_w(double d, double a) {
  const double b = 2.0 * kPi * d, den = a * a + b * b;
  if (den == 0.0) return 1.0;
  return 2.0 * (a + std::exp(-a / 2.0) * (b * std::sin(b / 2.0) - a * std::cos(b / 2.0))) / den;
}
double r_psi(double d, double a) {
  const double b = 2.0 * kPi * d, den = a * a + b * b;
  if (den == 0.0) return 1.0;
  return 2.0 * (std::exp(a / 2.0) * (b * std::sin(b / 2.0) + a * std::cos(b / 2.0)) - a) / den;
}
// diagonal of the truncated frame product at fractional lattice offset delta
double frame_diag(double delta, double a, double q) {
  const int K = (int)std::ceil(q) + 1;
  double acc = 0.0;
  for (int k = -K; k <= K; ++k) {
    const double d = (double)k - delta;
    if (std::fabs(d) < q) acc += r_psi(d, a) * r_w(d, a);
  }
  return acc;
}

// ---------------------------------------------------------------- ES kernel tables
double es(double z, double beta) {
  const double s = 1.0 - z * z;
  return s > 0.0 ? std::exp(beta * (std::sqrt(s) - 1.0)) : 0.0;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < (n + 1) / 2; ++i) {
    double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), pp = 0.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p2 = 0.0;
      for (int j = 1; j <= n; ++j) {
        const double p3 = p2;
        p2 = p1;
        p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
      }
      pp = n * (z * p1 - p2) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = -z;
    x[n - 1 - i] = z;
    w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// 1 / (continuous Fourier transform of the kernel) at the centred bins j - m/2 of a
// length-nfine periodic grid: phihat(j) = (W/2) int_{-1}^{1} es(z) cos(2 pi j (W/2) z / nfine) dz.
std::vector<double> deapod_table(int m, int nfine, int W, double beta) {
  std::vector<double> x, wq;
  gauss_legendre(std::max(200, 4 * W + 64), x, wq);
  std::vector<double> out(m);
  for (int jj = 0; jj < m; ++jj) {
    const double j = jj - m / 2;
    double acc = 0.0;
    for (size_t i = 0; i < x.size(); ++i)
      acc += wq[i] * es(x[i], beta) * std::cos(2.0 * kPi * j * (W / 2.0) * x[i] / nfine);
    out[jj] = 1.0 / ((W / 2.0) * acc);
  }
  return out;
}

// Two-level twiddle table of length-n transforms: [hi: exp(2 pi i 64 j / n), j < n/64]
// followed by [lo: exp(2 pi i l / n), l < 64], interleaved (re, im).
std::vector<double> twiddle_table(int n) {
  const int nh = n / 64;
  std::vector<double> tw(2 * (size_t)(nh + 64));
  for (int j = 0; j < nh; ++j) {
    tw[2 * j] = std::cos(2.0 * kPi * ((double)(64 * j) / n));
    tw[2 * j + 1] = std::sin(2.0 * kPi * ((double)(64 * j) / n));
  }
  for (int l = 0; l < 64; ++l) {
    tw[2 * (nh + l)] = std::cos(2.0 * kPi * ((double)l / n));
    tw[2 * (nh + l) + 1] = std::sin(2.0 * kPi * ((double)l / n));
  }
  return tw;
}

int log2_pow2_at_least(double v) {
  int l = 0;
  while ((double)(1 << l) < v - 1e-9) ++l;
  return l;
}

// ---------------------------------------------------------------- static scratch
// Device memory of tffr_entropy_step_noalloc: one array per GPU in the code object, so a
// call needs no allocation.  The array's host-side name is not a device address; the
// address is taken once per device (with that device current) by hipGetSymbolAddress
// and kept in scratch_addr[].
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[TFFR_SCRATCH_BYTES];
std::mutex scratch_mutex;
void* scratch_addr[kMaxDevices] = {};
hipError_t scratch_err[kMaxDevices] = {};
bool scratch_done[kMaxDevices] = {};

// Address of this device's scratch array (set up on the first call per device; the
// current device must be `dev`).  nullptr if the runtime could not resolve it.
void* scratch_for_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mutex);
  if (!scratch_done[dev]) {
    void* ptr = nullptr;
    scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    scratch_addr[dev] = scratch_err[dev] == hipSuccess ? ptr : nullptr;
    scratch_done[dev] = true;
  }
  return scratch_addr[dev];
}

// ---------------------------------------------------------------- plan
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

}  // namespace

struct tffr_plan {
  tffr_params prm;
  int device = 0;
  tffr::Geo geo{};
  int cb = 1;  // range columns per workgroup in the azimuth stage
  int ffr_halfband = 0;
  int ffr_route = 0;  // plain FFR: 0 selected inversion of the frame product, 1 of Sa Sb
  int ffr_lmax = 0;   // plain FFR: most lattice points of a slice
  int ffr_nwg = 0;    // plain FFR: workgroups of the solve (each with its own scratch)
  int ffr_status = 0; // plain FFR: outcome of the plan-time solve (0 ok, 1 pivot, 3 conditioning, 2 lattice)
  bool from_xy = false;      // made from explicit coordinates (no Stolt map)
  std::vector<double> hku;   // azimuth wavenumbers (host copy)
  int stolt_part = 0;        // Stolt baseline: samples per part (span below mx - 1 lattice units)
  double beta = 0.0;
  // device tables
  DevBuf k, ku, kx, ky, ystart, ytap, deapx, deapy, twx, twy, poly, ffr_d, ycn, ycw, deapf;
  int logfg = 0;           // front end with position errors: log2 of its periodic grid (>= 2 n_pulses)
  DevBuf fpos;             // its source positions on that grid (FP64), refreshed by every call
  size_t fpos_n = 0;
  // workspace layout
  bool ent_fused = false;  // entropy step uses the fused azimuth kernel
  int coord_cb = 0;        // azimuth block width of the coordinate-gradient kernels (0: unsupported)
  void* scratch = nullptr;  // this device's static scratch array (tffr_entropy_step_noalloc)
  size_t step_bytes = 0;    // workspace bytes tffr_entropy_step reads and writes
  size_t off_hx = 0, off_h12 = 0, off_cblk = 0, off_part = 0, off_stats = 0, off_kept = 0, off_count = 0, off_status = 0, off_gband = 0, off_zband = 0,
         off_dband = 0, work_bytes = 0;
  bool dbl() const { return prm.dtype == TFFR_C128; }
  size_t csize() const { return dbl() ? 16 : 8; }
  size_t rsize() const { return dbl() ? 8 : 4; }
};

namespace {

tffr_status hip_status(hipError_t e) { return e == hipSuccess ? TFFR_OK : TFFR_ERR_HIP; }

template <typename T>
tffr_status upload(DevBuf& b, const std::vector<T>& v) {
  if (v.empty()) return TFFR_OK;
  if (hipMalloc(&b.p, v.size() * sizeof(T)) != hipSuccess) return TFFR_ERR_NOMEM;
  return hip_status(hipMemcpy(b.p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
}

template <typename R>
std::vector<R> cast(const std::vector<double>& v) {
  return std::vector<R>(v.begin(), v.end());
}

template <typename R>
tffr::Tab<R> tables(const tffr_plan* P) {
  tffr::Tab<R> t;
  t.k = (const double*)P->k.p;
  t.ku = (const double*)P->ku.p;
  t.kx = (const double*)P->kx.p;
  t.ky = (const R*)P->ky.p;
  t.ystart = (const int32_t*)P->ystart.p;
  t.ytap = (const R*)P->ytap.p;
  t.deapx = (const R*)P->deapx.p;
  t.deapy = (const R*)P->deapy.p;
  t.twx = (const cplx<R>*)P->twx.p;
  t.twy = (const cplx<R>*)P->twy.p;
  t.poly = (const float*)P->poly.p;
  t.deapf = (const R*)P->deapf.p;
  t.ycell_n = (const int32_t*)P->ycn.p;
  t.ycell_w = (const R*)P->ycw.p;
  return t;
}

int sample_type(const tffr_plan* P) {
  return P->prm.dtype == TFFR_C128 ? tffr::ST_C128 : (P->prm.dtype == TFFR_C64_FP16IN ? tffr::ST_H2 : tffr::ST_C64);
}

// Piecewise polynomial of 1/g(delta) on (0, 1) for the FP32 path: nseg segments, local
// variable t in [-1, 1], monomial coefficients (highest first) from interpolation at
// Chebyshev points, stored coefficient-major (out[j * nseg + s]: lanes evaluating
// different segments read consecutive words, so distinct LDS banks).  Returns false
// when the fit misses 2e-8 relative somewhere.
bool fit_weight_poly(double a, double q, int nseg, int deg, std::vector<float>& out) {
  out.assign((size_t)nseg * (deg + 1), 0.0f);
  const int np = deg + 1;
  std::vector<double> tn(np), fv(np), A((size_t)np * np), c(np);
  for (int s = 0; s < nseg; ++s) {
    for (int i = 0; i < np; ++i) {
      tn[i] = std::cos(kPi * (2.0 * i + 1.0) / (2.0 * np));
      const double delta = (s + 0.5 * (tn[i] + 1.0)) / nseg;
      fv[i] = 1.0 / frame_diag(delta, a, q);
      for (int j = 0; j < np; ++j) A[(size_t)i * np + j] = std::pow(tn[i], deg - j);
    }
    // Gaussian elimination with partial pivoting on the small Vandermonde system
    std::vector<double> M(A), rhs(fv);
    for (int col = 0; col < np; ++col) {
      int piv = col;
      for (int r = col + 1; r < np; ++r)
        if (std::fabs(M[(size_t)r * np + col]) > std::fabs(M[(size_t)piv * np + col])) piv = r;
      for (int j = 0; j < np; ++j) std::swap(M[(size_t)col * np + j], M[(size_t)piv * np + j]);
      std::swap(rhs[col], rhs[piv]);
      for (int r = col + 1; r < np; ++r) {
        const double l = M[(size_t)r * np + col] / M[(size_t)col * np + col];
        for (int j = col; j < np; ++j) M[(size_t)r * np + j] -= l * M[(size_t)col * np + j];
        rhs[r] -= l * rhs[col];
      }
    }
    for (int r = np - 1; r >= 0; --r) {
      double v = rhs[r];
      for (int j = r + 1; j < np; ++j) v -= M[(size_t)r * np + j] * c[j];
      c[r] = v / M[(size_t)r * np + r];
    }
    for (int j = 0; j < np; ++j) out[(size_t)j * nseg + s] = (float)c[j];
    for (int i = 0; i <= 32; ++i) {
      const double t = -1.0 + i / 16.0, delta = (s + 0.5 * (t + 1.0)) / nseg;
      if (delta <= 0.0 || delta >= 1.0) continue;
      double v = 0.0;
      for (int j = 0; j < np; ++j) v = v * t + c[j];
      const double ex = 1.0 / frame_diag(delta, a, q);
      if (std::fabs(v - ex) > 2e-8 * std::fabs(ex)) return false;
    }
  }
  return true;
}

// Range wavenumber of sample (n, i) on the host: the Stolt map of (k, ku), or the
// explicit table of a plan made from coordinates.  Same operation order as the kernels.
struct HostKx {
  const double* k;
  const double* ku;
  const double* kx;
  int n_freq;
  double operator()(int n, int i) const {
    return kx ? kx[(size_t)n * n_freq + i] : std::sqrt(4.0 * (k[i] * k[i]) - ku[n] * ku[n]);
  }
};

tffr_status check_params(const tffr_params* p) {
  if (!p) return TFFR_ERR_ARG;
  if (p->n_pulses < 1 || p->n_freq < 1) return TFFR_ERR_ARG;
  if (p->mx < 2 || p->my < 2 || (p->mx & 1) || (p->my & 1)) return TFFR_ERR_ARG;
  if (p->mx > (1 << kMaxLogN) || p->my > (1 << kMaxLogN)) return TFFR_ERR_UNSUPPORTED;
  if (!(p->fov_x > 0.0) || !(p->fov_y > 0.0) || !std::isfinite(p->fov_x) || !std::isfinite(p->fov_y))
    return TFFR_ERR_ARG;
  if (p->weighting < TFFR_W_NONE || p->weighting > TFFR_W_USER) return TFFR_ERR_ARG;
  if (!(p->window_a >= 0.0) || !std::isfinite(p->window_a)) return TFFR_ERR_ARG;
  if (!(p->q >= 1.0) || !(p->q <= 64.0)) return TFFR_ERR_ARG;
  if (p->band_r < 0 || p->band_r > 8) return TFFR_ERR_ARG;
  if (!(p->tau > 0.0) || !std::isfinite(p->tau)) return TFFR_ERR_ARG;
  if (p->thresh_mode != TFFR_THRESH_LITERAL && p->thresh_mode != TFFR_THRESH_CORRELATION) return TFFR_ERR_ARG;
  if (p->kernel_width < 2 || p->kernel_width > 16) return TFFR_ERR_UNSUPPORTED;
  if (!(p->upsampfac >= 1.25) || !(p->upsampfac <= 4.0)) return TFFR_ERR_UNSUPPORTED;
  if (p->dtype != TFFR_C64 && p->dtype != TFFR_C128 && p->dtype != TFFR_C64_FP16IN) return TFFR_ERR_UNSUPPORTED;
  const int lx = log2_pow2_at_least(p->upsampfac * p->mx), ly = log2_pow2_at_least(p->upsampfac * p->my);
  if (std::max(lx, 6) > kMaxLogN || std::max(ly, 6) > kMaxLogN) return TFFR_ERR_UNSUPPORTED;
  if (p->gridding != TFFR_GRID_ES && p->gridding != TFFR_GRID_LITERAL) return TFFR_ERR_ARG;
  if (p->gridding == TFFR_GRID_LITERAL) {
    // the image lattice is the range grid: a power of two the LDS FFT handles; 2q taps
    if (p->q != std::floor(p->q) || p->q > 8.0) return TFFR_ERR_UNSUPPORTED;
    if (p->mx < 64 || (p->mx & (p->mx - 1))) return TFFR_ERR_UNSUPPORTED;
  }
  return TFFR_OK;
}

// Half bandwidth of the frame product: the largest |p - p'| whose windows
// (lam - q, lam + q) share an integer, over all slices (plus one for rounding).
int ffr_halfband(const tffr_params* p, const HostKx& kx) {
  int b = 0;
  std::vector<double> lam(p->n_freq);
  for (int n = 0; n < p->n_pulses; ++n) {
    for (int i = 0; i < p->n_freq; ++i) lam[i] = kx(n, i) * p->fov_x / (2.0 * kPi);
    int j = 0;
    for (int i = 0; i < p->n_freq; ++i) {
      const double top = std::ceil(lam[i] + p->q) - 1.0;  // largest integer < lam + q
      if (j < i) j = i;
      while (j + 1 < p->n_freq && std::floor(lam[j + 1] - p->q) + 1.0 <= top) ++j;
      b = std::max(b, j - i);
    }
  }
  return b + 1;
}

// Plain-FFR route (see tffr_ffr.hip).  Route 0: every slice has no more samples than
// lattice points (the frame product can have full rank) and its half-band, widened to r,
// is at most 8: selected inversion of the product itself.  Route 1: every slice has more
// samples than lattice points (rank-deficient product, full-rank factors), q <= 3 and
// r times the largest sample spacing plus 2q at most 10 (the lattice offsets the band of
// D reaches within the half-band 10 of Sa Sb): selected inversion of Sa Sb.  Anything
// else is TFFR_ERR_UNSUPPORTED.  lmax: the most lattice points of a slice.
constexpr int kFfrDirectMaxBand = 8;
constexpr int kFfrNormalBand = 10;
tffr_status ffr_route(const tffr_params* p, const HostKx& kx, int* route, int* hb_out, int* lmax_out) {
  const int P = p->n_freq;
  int n_full = 0, n_def = 0, lmax = 0;
  double spmax = 0.0;
  std::vector<double> lam(P);
  for (int n = 0; n < p->n_pulses; ++n) {
    for (int i = 0; i < P; ++i) lam[i] = kx(n, i) * p->fov_x / (2.0 * kPi);
    for (int i = 0; i + 1 < P; ++i) spmax = std::max(spmax, lam[i + 1] - lam[i]);
    const int l0 = (int)std::floor(lam[0] - p->q) + 1;
    const int L = (int)(std::ceil(lam[P - 1] + p->q) - 1.0) - l0 + 1;
    lmax = std::max(lmax, L);
    if (P <= L) ++n_full; else ++n_def;
  }
  const int hb = ffr_halfband(p, kx);
  *hb_out = hb;
  *lmax_out = lmax + 2;  // margin: the kernels round the lattice coordinate in their own order
  if (p->q > 4.0) return TFFR_ERR_UNSUPPORTED;  // at most 2 (ceil(q) + 1) + 1 = 11 lattice taps
  if (n_def == 0 && std::max(hb, p->band_r) <= kFfrDirectMaxBand) {
    *route = 0;
    return TFFR_OK;
  }
  if (n_full == 0 && p->q <= 3.0 && p->band_r * spmax + 2.0 * p->q <= (double)kFfrNormalBand) {
    *route = 1;
    return TFFR_OK;
  }
  return TFFR_ERR_UNSUPPORTED;
}

}  // namespace

namespace {

template <typename R>
tffr_status do_forward(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw, void* img,
                       void* work, hipStream_t st, int stage_only) {
  const tffr::Tab<R> t = tables<R>(P);
  const R* w = (const R*)uw;
  if (!w && P->prm.weighting == TFFR_W_FFR) w = (const R*)P->ffr_d.p;
  cplx<R>* hx = (cplx<R>*)((char*)work + P->off_hx);
  if (stage_only >= 0)
    return hip_status(tffr::launch_fwd_rows<R>(P->geo, t, sample_type(P), smp, (const R*)ph, (const R*)da, w,
                                               (cplx<R>*)img, stage_only, st));
  hipError_t e = tffr::launch_fwd_rows<R>(P->geo, t, sample_type(P), smp, (const R*)ph, (const R*)da, w, hx, 1, st);
  if (e == hipSuccess) e = tffr::launch_fwd_cols<R>(P->geo, t, P->cb, hx, (cplx<R>*)img, nullptr, st);
  return hip_status(e);
}

template <typename R>
tffr_status do_stolt(tffr_plan* P, const void* smp, const void* ph, const void* da, void* img, void* work,
                     hipStream_t st) {
  const tffr::Tab<R> t = tables<R>(P);
  cplx<R>* hx = (cplx<R>*)((char*)work + P->off_hx);
  hipError_t e = tffr::launch_stolt_rows<R>(P->geo, t, sample_type(P), smp, (const R*)ph, (const R*)da,
                                            P->stolt_part, hx, st);
  if (e == hipSuccess) e = tffr::launch_fwd_cols<R>(P->geo, t, P->cb, hx, (cplx<R>*)img, nullptr, st);
  return hip_status(e);
}

template <typename R>
tffr_status do_adjoint(tffr_plan* P, const void* cot, const void* smp, const void* ph, const void* da, const void* uw,
                       void* gs, void* gph, void* gda, void* work, hipStream_t st) {
  const tffr::Tab<R> t = tables<R>(P);
  const R* w = (const R*)uw;
  if (!w && P->prm.weighting == TFFR_W_FFR) w = (const R*)P->ffr_d.p;
  cplx<R>* hx = (cplx<R>*)((char*)work + P->off_hx);
  hipError_t e = tffr::launch_adj_cols<R>(P->geo, t, P->cb, (const cplx<R>*)cot, hx, nullptr, nullptr, 0, nullptr, st);
  if (e == hipSuccess)
    e = tffr::launch_adj_rows<R>(P->geo, t, sample_type(P), hx, smp, (const R*)ph, (const R*)da, w, (cplx<R>*)gs,
                                 (R*)gph, (R*)gda, tffr::EntComb<R>{}, st);
  return hip_status(e);
}

// The entropy step's range adjoint on the fields in the workspace (see tffr_debug.h).
template <typename R>
hipError_t launch_ent_adj_rows(tffr_plan* P, const void* smp, const void* ph, const void* da, const R* w,
                               double* loss, void* gs, void* gph, void* gda, void* work, hipStream_t st) {
  char* wb = (char*)work;
  const int nparts = (P->prm.mx + P->cb - 1) / P->cb;
  tffr::EntComb<R> ec{};
  ec.h12 = (const cplx<R>*)(wb + P->off_h12);
  ec.cblk = (const R*)(wb + P->off_cblk);
  ec.cb = P->cb;
  if (nparts <= kFuseStatsMax) {
    ec.partials = (const double*)(wb + P->off_part);
    ec.nparts = nparts;
    ec.loss = loss;
  } else {
    ec.stats = (const double*)(wb + P->off_stats);
  }
  return tffr::launch_adj_rows<R>(P->geo, tables<R>(P), sample_type(P), (const cplx<R>*)(wb + P->off_hx), smp,
                                  (const R*)ph, (const R*)da, w, (cplx<R>*)gs, (R*)gph, (R*)gda, ec, st);
}

// The step's launches in order; with `mark` non-null, mark(i) runs before launch i and
// mark(nk) after the last (per-launch timing), and *nk receives the number of launches.
// Launch number `dup` is issued twice (marginal timing; every launch of the step writes
// its outputs without accumulating, so a repeat leaves them as one launch would).
template <typename R>
tffr_status do_entropy_step(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw, void* img,
                            double* loss, void* gs, void* gph, void* gda, void* work, hipStream_t st,
                            hipError_t (*mark)(void*, int) = nullptr, void* mark_ctx = nullptr, int* nk = nullptr,
                            int dup = -1) {
  const tffr::Tab<R> t = tables<R>(P);
  const R* w = (const R*)uw;
  if (!w && P->prm.weighting == TFFR_W_FFR) w = (const R*)P->ffr_d.p;
  char* wb = (char*)work;
  cplx<R>* hx = (cplx<R>*)(wb + P->off_hx);
  double* part = (double*)(wb + P->off_part);
  double* stats = (double*)(wb + P->off_stats);
  const int nparts = (P->prm.mx + P->cb - 1) / P->cb;
  cplx<R>* h12 = (cplx<R>*)(wb + P->off_h12);
  R* cblk = (R*)(wb + P->off_cblk);
  int k = 0;
  // launch number k of the step: mark, launch (twice if k == dup)
  auto issue = [&](hipError_t e, auto&& launch) -> hipError_t {
    if (e == hipSuccess && mark) e = mark(mark_ctx, k);
    if (e == hipSuccess) e = launch();
    if (e == hipSuccess && k == dup) e = launch();
    ++k;
    return e;
  };
  // range stage; azimuth forward + entropy sums + adjoint azimuth transforms of the two
  // gradient fields in one kernel (written interleaved); range
  // adjoint combining the fields with the global entropy sums
  hipError_t e = issue(hipSuccess, [&] {
    return tffr::launch_fwd_rows<R>(P->geo, t, sample_type(P), smp, (const R*)ph, (const R*)da, w, hx, 1, st);
  });
  // few partial sums: every adjoint block reduces them itself (no separate launch)
  const bool fuse = nparts <= kFuseStatsMax;
  auto stats_launch = [&] { return tffr::launch_entropy_stats(part, nparts, stats, loss, st); };
  if (!P->ent_fused) {  // image round trip: forward azimuth stage, then the adjoint one
    e = issue(e, [&] { return tffr::launch_fwd_cols<R>(P->geo, t, P->cb, hx, (cplx<R>*)img, part, st); });
    if (!fuse) e = issue(e, stats_launch);
    e = issue(e, [&] {
      return fuse ? tffr::launch_adj_cols<R>(P->geo, t, P->cb, (const cplx<R>*)img, hx, nullptr, part, nparts, loss, st)
                  : tffr::launch_adj_cols<R>(P->geo, t, P->cb, (const cplx<R>*)img, hx, stats, nullptr, 0, nullptr, st);
    });
    e = issue(e, [&] {
      return tffr::launch_adj_rows<R>(P->geo, t, sample_type(P), hx, smp, (const R*)ph, (const R*)da, w,
                                      (cplx<R>*)gs, (R*)gph, (R*)gda, tffr::EntComb<R>{}, st);
    });
  } else {
    e = issue(e, [&] { return tffr::launch_ent_cols<R>(P->geo, t, P->cb, hx, (cplx<R>*)img, part, cblk, h12, st); });
    if (!fuse) e = issue(e, stats_launch);
    e = issue(e, [&] { return launch_ent_adj_rows<R>(P, smp, ph, da, w, loss, gs, gph, gda, work, st); });
  }
  if (e == hipSuccess && mark) e = mark(mark_ctx, k);
  if (nk) *nk = k;
  return hip_status(e);
}

// Launch names of the step, in order, for tffr_debug_step_kernel_times.
int step_kernel_names(const tffr_plan* P, const char** names) {
  const int nparts = (P->prm.mx + P->cb - 1) / P->cb;
  int k = 0;
  names[k++] = P->geo.range_mode == 1 ? "k_fwd_rows_run" : "k_fwd_rows";
  if (!P->ent_fused) {
    names[k++] = "k_fwd_cols";
    if (nparts > kFuseStatsMax) names[k++] = "k_entropy_stats";
    names[k++] = "k_adj_cols";
  } else {
    names[k++] = "k_ent_cols";
    if (nparts > kFuseStatsMax) names[k++] = "k_entropy_stats";
  }
  names[k++] = "k_adj_rows";
  return k;
}

struct EventMarks {
  hipEvent_t ev[8];
  hipStream_t st;
};
hipError_t record_mark(void* ctx, int i) {
  EventMarks* m = (EventMarks*)ctx;
  return hipEventRecord(m->ev[i], m->st);
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// Range gridding schedule (see k_fwd_rows, k_fwd_rows_run).  U = kx fov_x nfx / (2 pi mx)
// is a sample's unwrapped fine cell coordinate.  S (samples per thread run / per sub-pass group) satisfies
// S * (smallest spacing of U) > W + 1, one cell of margin over the W-cell tap span, so
// the taps of samples S apart never meet even when a fraction rounds across a cell
// boundary.  Slices are cut into parts whose span (plus taps) stays inside the fine row, so
// after wrapping two samples of a part never share cells.  The run kernel (mode 1) serves
// every plan with W <= kRunWindow and kernel gridding, dense or sparse; each of its
// threads takes at most one run per part.  The sub-pass kernel (mode 0) serves wider
// kernels and the literal lattice taps.

void range_schedule(const tffr_params* p, const HostKx& kx, int nfx, int W, int nt, int* S, int* part_len,
                    int* mode, int* pair) {
  const double tx = p->fov_x / (2.0 * kPi * p->mx);
  const int P = p->n_freq;
  double smin = 1e300, smax = 0.0;
  int Q = 1;
  std::vector<double> U(P);
  for (int n = 0; n < p->n_pulses; ++n) {
    for (int i = 0; i < P; ++i) U[i] = kx(n, i) * tx * nfx;
    for (int i = 0; i + 1 < P; ++i) {
      smin = std::min(smin, U[i + 1] - U[i]);
      smax = std::max(smax, U[i + 1] - U[i]);
    }
    for (;; ++Q) {
      const int len = (P + Q - 1) / Q;
      bool ok = true;
      for (int a = 0; a < P && ok; a += len) {
        const int b = std::min(a + len, P) - 1;
        ok = (U[b] - U[a] + W + 2.0) <= (double)nfx;
      }
      if (ok) break;
    }
  }
  int s = 1;
  if (P > 1) {
    const double sm = smin * (1.0 - 1e-9);
    s = (int)std::min<double>((double)P, std::floor((W + 1.0) / sm) + 1.0);
  }
  *S = std::max(1, s);
  int m = (P > 1 && W <= tffr::kRunWindow) ? 1 : 0;
  if (p->gridding == TFFR_GRID_LITERAL) m = 0;  // lattice taps: sub-pass kernel only
  else if (const char* e = std::getenv("TFFR_RANGE_MODE")) {
    const int v = std::atoi(e);
    if (v == 0 || (v == 1 && W <= tffr::kRunWindow)) m = v;
  }
  *mode = m;
  // on complex64 rows of 4096 cells and more with samples under half a cell apart (so two
  // consecutive samples' first cells differ by at most one) the run kernel takes its
  // samples two at a time, summing both samples' taps in registers over W + 1 cells; then
  // samples S - 1 apart must keep the same clearance
  *pair = (m == 1 && W == 7 && P > 1 && p->dtype != TFFR_C128 && nfx >= 4096 && smax < 0.5) ? 1 : 0;
  if (*pair) *S = std::min(P, *S + 1);
  int len = (P + Q - 1) / Q;
  if (m == 1) len = std::min(len, nt * *S);
  *part_len = len;
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

void tffr_default_params(tffr_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->weighting = TFFR_W_TFFR;
  p->window_a = 0.01;
  p->q = 3.0;
  p->band_r = 2;
  p->tau = 0.97;
  p->thresh_mode = TFFR_THRESH_LITERAL;
  p->kernel_width = 7;
  p->upsampfac = 2.0;
  p->dtype = TFFR_C64;
  p->gridding = TFFR_GRID_ES;
}

const char* tffr_status_string(tffr_status s) {
  switch (s) {
    case TFFR_OK: return "TFFR_OK";
    case TFFR_ERR_ARG: return "TFFR_ERR_ARG: invalid argument";
    case TFFR_ERR_EVANESCENT: return "TFFR_ERR_EVANESCENT: 4 k^2 <= ku^2 for some sample";
    case TFFR_ERR_NONMONOTONE: return "TFFR_ERR_NONMONOTONE: k is not strictly increasing";
    case TFFR_ERR_LAYOUT: return "TFFR_ERR_LAYOUT: buffer layout or size mismatch";
    case TFFR_ERR_UNSUPPORTED: return "TFFR_ERR_UNSUPPORTED: configuration not supported";
    case TFFR_ERR_SINGULAR: return "TFFR_ERR_SINGULAR: plain-FFR solve is numerically singular in FP64";
    case TFFR_ERR_NOMEM: return "TFFR_ERR_NOMEM: allocation failed";
    case TFFR_ERR_HIP: return "TFFR_ERR_HIP: HIP runtime error";
    case TFFR_ERR_SCRATCH: return "TFFR_ERR_SCRATCH: the problem needs more than the static scratch array holds";
  }
  return "TFFR_ERR_UNKNOWN";
}

tffr_status tffr_validate(const tffr_params* p, const double* k, const double* ku) {
  tffr_status s = check_params(p);
  if (s != TFFR_OK) return s;
  if (!k || !ku) return TFFR_ERR_ARG;
  for (int i = 0; i < p->n_freq; ++i)
    if (!std::isfinite(k[i])) return TFFR_ERR_ARG;
  for (int i = 0; i < p->n_pulses; ++i)
    if (!std::isfinite(ku[i])) return TFFR_ERR_ARG;
  for (int i = 1; i < p->n_freq; ++i)
    if (!(k[i] > k[i - 1])) return TFFR_ERR_NONMONOTONE;
  double kmin = std::fabs(k[0]), kumax = 0.0;
  for (int i = 0; i < p->n_freq; ++i) kmin = std::min(kmin, std::fabs(k[i]));
  for (int i = 0; i < p->n_pulses; ++i) kumax = std::max(kumax, std::fabs(ku[i]));
  if (!(4.0 * (kmin * kmin) - kumax * kumax > 0.0)) return TFFR_ERR_EVANESCENT;
  if (p->weighting == TFFR_W_FFR) {
    int route, hb, lmax;
    return ffr_route(p, HostKx{k, ku, nullptr, p->n_freq}, &route, &hb, &lmax);
  }
  return TFFR_OK;
}

tffr_status tffr_validate_xy(const tffr_params* p, const double* kx, const double* ky) {
  tffr_status s = check_params(p);
  if (s != TFFR_OK) return s;
  if (!kx || !ky) return TFFR_ERR_ARG;
  const size_t nf = (size_t)p->n_freq;
  for (size_t i = 0; i < (size_t)p->n_pulses * nf; ++i)
    if (!std::isfinite(kx[i]) || !std::isfinite(ky[i])) return TFFR_ERR_ARG;
  for (int n = 0; n < p->n_pulses; ++n) {
    const double* r = kx + n * nf;
    const double* y = ky + n * nf;
    for (size_t i = 1; i < nf; ++i) {
      if (y[i] != y[0]) return TFFR_ERR_LAYOUT;
      if (!(r[i] > r[i - 1])) return TFFR_ERR_NONMONOTONE;
    }
  }
  if (p->weighting == TFFR_W_FFR) {
    int route, hb, lmax;
    return ffr_route(p, HostKx{nullptr, nullptr, kx, p->n_freq}, &route, &hb, &lmax);
  }
  return TFFR_OK;
}

}  // extern "C"

namespace {

// Plan from (k, ku) (Stolt map in the kernels) or from explicit coordinates (kx_tab
// non-null; ku then holds each slice's ky).
tffr_status plan_create(const tffr_params* p, const double* k, const double* ku, const double* kx_tab,
                        tffr_plan** out) {
  tffr_status s = TFFR_OK;
  tffr_plan* P = new (std::nothrow) tffr_plan();
  if (!P) return TFFR_ERR_NOMEM;
  P->prm = *p;
  auto fail = [&](tffr_status e) {
    delete P;
    return e;
  };
  if (hipGetDevice(&P->device) != hipSuccess) return fail(TFFR_ERR_HIP);

  const int W = p->kernel_width;
  const bool lit = p->gridding == TFFR_GRID_LITERAL;
  // range grid: the oversampled ES grid, or the image lattice itself (literal Algorithm 1)
  const int lognx = lit ? log2_pow2_at_least(p->mx) : std::max(6, log2_pow2_at_least(p->upsampfac * p->mx));
  const int logny = std::max(6, log2_pow2_at_least(p->upsampfac * p->my));
  const int nfx = 1 << lognx, nfy = 1 << logny;
  // ES shape for the achieved upsampling factor: beta = 2.30 W at sigma = 2, scaled
  // for other sigma with the usual (1 - 1/(2 sigma)) law.
  const double sig = lit ? (double)nfy / p->my : std::min((double)nfx / p->mx, (double)nfy / p->my);
  P->beta = 2.30 * W * (1.0 - 1.0 / (2.0 * sig)) / 0.75;
  const size_t csz = P->csize();
  const size_t lds_max = tffr::max_dynamic_lds();
  const size_t twx_n = nfx / 64 + 64, twy_n = nfy / 64 + 64;
  if ((nfx + twx_n) * csz + 2048 + (p->weighting == TFFR_W_FFR ? (size_t)p->n_freq * csz : 0) > lds_max ||
      (nfy + twy_n) * csz > lds_max || (nfy + (size_t)p->n_pulses + twy_n) * csz > lds_max)
    return fail(TFFR_ERR_UNSUPPORTED);
  // range columns per workgroup in the azimuth stage: keep the forward kernel's LDS
  // (columns + staged spectra + twiddles) within 64 KB where possible, and at least
  // ~512 workgroups in flight
  auto cols_lds = [&](int c) { return ((size_t)nfy + p->n_pulses) * c * csz + twy_n * csz; };
  int cb = 4;
  while (cb > 1 && cols_lds(cb) > 65536) cb >>= 1;
  while (cb > 1 && (p->mx + cb - 1) / cb < 512) cb >>= 1;
  if (const char* e = std::getenv("TFFR_AZ_COLS")) {
    const int v = std::atoi(e);
    if ((v == 1 || v == 2 || v == 4) && cols_lds(v) <= lds_max) cb = v;
  }
  P->cb = cb;
  // entropy step: the fused azimuth kernel holds [CB][nfy] image columns plus, in the
  // staged-spectra space, at least [CB][nfy] more
  P->ent_fused = ((size_t)nfy * cb + std::max<size_t>((size_t)p->n_pulses * cb, (size_t)nfy * cb) + twy_n) * csz <=
                 lds_max;
  if (const char* e = std::getenv("TFFR_ENT_FUSED"))  // 0: force the image round trip
    if (std::atoi(e) == 0) P->ent_fused = false;
  // coordinate gradients: two fields per fine row / column in LDS
  if ((2 * (size_t)nfx + twx_n) * csz + 2048 <= lds_max)
    for (int c = cb; c >= 1 && !P->coord_cb; c >>= 1)
      if ((2 * (size_t)nfy * c + twy_n) * csz <= lds_max) P->coord_cb = c;

  tffr::Geo& g = P->geo;
  g.n_pulses = p->n_pulses;
  g.n_freq = p->n_freq;
  g.mx = p->mx;
  g.my = p->my;
  g.nfx = nfx;
  g.nfy = nfy;
  g.lognfx = lognx;
  g.lognfy = logny;
  g.W = W;
  g.literal = lit ? 1 : 0;
  g.lit_taps = lit ? 2 * (int)p->q : 0;
  g.weighting = p->weighting;
  g.thresh_mode = p->thresh_mode;
  g.band_r = p->band_r;
  g.beta = P->beta;
  g.tx_scale = p->fov_x / (2.0 * kPi * p->mx);
  g.fov_x = p->fov_x;
  g.fov_y = p->fov_y;
  g.a = p->window_a;
  g.q = p->q;
  g.tau = p->tau;
  g.ema2 = std::exp(-p->window_a / 2.0);
  g.epa2 = std::exp(p->window_a / 2.0);
  const double g0 = frame_diag(0.0, p->window_a, p->q);
  g.inv_g0 = g0 != 0.0 ? 1.0 / g0 : 0.0;
  g.keep0 = p->thresh_mode == TFFR_THRESH_LITERAL ? (std::fabs(g.inv_g0) >= p->tau) : (g0 >= p->tau);
  g.near_rel = 1e-5;
  g.near_f = (float)g.near_rel;
  g.thr_f = (float)(p->thresh_mode == TFFR_THRESH_LITERAL ? p->tau : 1.0 / p->tau);

  std::vector<double> kv, kuv(ku, ku + p->n_pulses), kxv;
  if (kx_tab)
    kxv.assign(kx_tab, kx_tab + (size_t)p->n_pulses * p->n_freq);
  else
    kv.assign(k, k + p->n_freq);
  // per-slice azimuth taps
  std::vector<int32_t> ys(p->n_pulses);
  std::vector<double> taps((size_t)p->n_pulses * W);
  for (int n = 0; n < p->n_pulses; ++n) {
    const double t = ku[n] * p->fov_y / (2.0 * kPi * p->my);
    const double u = (t - std::floor(t)) * nfy;
    const double ui = std::floor(u), f = u - ui;
    const int k0 = (int)std::ceil(f - W / 2.0);
    ys[n] = (int32_t)ui + k0;
    for (int i = 0; i < W; ++i) taps[(size_t)n * W + i] = es((k0 + i - f) / (W / 2.0), P->beta);
  }
  // azimuth cell table: for every fine azimuth cell, the (slice, tap) pairs that reach it,
  // padded to the largest count with (slice 0, tap 0)
  std::vector<int32_t> ccount(nfy, 0);
  for (int n = 0; n < p->n_pulses; ++n)
    for (int i = 0; i < W; ++i) ccount[(((ys[n] + i) % nfy) + nfy) % nfy]++;
  const int yemax = std::max(1, *std::max_element(ccount.begin(), ccount.end()));
  std::vector<int32_t> cn((size_t)nfy * yemax, 0);
  std::vector<double> cw((size_t)nfy * yemax, 0.0);
  std::fill(ccount.begin(), ccount.end(), 0);
  for (int n = 0; n < p->n_pulses; ++n)
    for (int i = 0; i < W; ++i) {
      const int cell = (((ys[n] + i) % nfy) + nfy) % nfy;
      const size_t slot = (size_t)(ccount[cell]++) * nfy + cell;
      cn[slot] = n;
      cw[slot] = taps[(size_t)n * W + i];
    }
  g.yemax = yemax;
  const HostKx hkx{k, ku, kx_tab, p->n_freq};
  range_schedule(p, hkx, nfx, lit ? 2 * (int)p->q : W, tffr::rows_threads(lognx), &g.sub, &g.part_len,
                 &g.range_mode, &g.run_pair);
  {
    // slices of several parts on rows of at most 4096 cells, where one workgroup per slice
    // leaves fewer than four waves per SIMD: two parts at once, on twice the threads, each
    // into its own LDS row (the rows are summed before the FFT).  That halves each lane's
    // chain of dependent read-add-writes; on a full chip the idle half of an odd last part
    // costs more than it saves.
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess || ncu < 1)
      ncu = 256;
    const int nparts = (p->n_freq + g.part_len - 1) / g.part_len;
    const int nt = tffr::rows_threads(lognx);
    const bool sparse_chip = (double)p->n_pulses * (nt / 64) < 4.0 * 4.0 * ncu;
    g.run_parts = (g.range_mode == 1 && !g.run_pair && nparts >= 2 && lognx <= 12 && 2 * nt <= 1024 && sparse_chip)
                      ? 2
                      : 1;
    if (const char* e = std::getenv("TFFR_RUN_PARTS")) {
      const int v = std::atoi(e);
      if (v == 1) g.run_parts = 1;
      if (v == 2 && g.range_mode == 1 && !g.run_pair && lognx <= 12 && 2 * nt <= 1024) g.run_parts = 2;
    }
  }
  std::vector<double> dx = deapod_table(p->mx, nfx, W, P->beta), dy = deapod_table(p->my, nfy, W, P->beta);
  // front end with position errors: a grid of at least twice the azimuth bins
  P->logfg = 6;
  while ((1 << P->logfg) < 2 * p->n_pulses) ++P->logfg;
  const std::vector<double> df = deapod_table(p->n_pulses, 1 << P->logfg, W, P->beta);
  if (lit)  // divide by the window w(u) = exp(-a |u|), u = X / fov_x (Algorithm 1)
    for (int j = 0; j < p->mx; ++j) dx[j] = std::exp(p->window_a * std::fabs((j - p->mx / 2) / (double)p->mx));
  std::vector<double> twx = twiddle_table(nfx), twy = twiddle_table(nfy);
  if (P->dbl()) {
    s = upload(P->ky, kuv);
    if (s == TFFR_OK) s = upload(P->ycw, cw);
    if (s == TFFR_OK) s = upload(P->ytap, taps);
    if (s == TFFR_OK) s = upload(P->deapx, dx);
    if (s == TFFR_OK) s = upload(P->deapy, dy);
    if (s == TFFR_OK) s = upload(P->deapf, df);
    if (s == TFFR_OK) s = upload(P->twx, twx);
    if (s == TFFR_OK) s = upload(P->twy, twy);
  } else {
    s = upload(P->ky, cast<float>(kuv));
    if (s == TFFR_OK) s = upload(P->ycw, cast<float>(cw));
    if (s == TFFR_OK) s = upload(P->ytap, cast<float>(taps));
    if (s == TFFR_OK) s = upload(P->deapx, cast<float>(dx));
    if (s == TFFR_OK) s = upload(P->deapy, cast<float>(dy));
    if (s == TFFR_OK) s = upload(P->deapf, cast<float>(df));
    if (s == TFFR_OK) s = upload(P->twx, cast<float>(twx));
    if (s == TFFR_OK) s = upload(P->twy, cast<float>(twy));
  }
  if (s == TFFR_OK) s = upload(P->k, kv);
  if (s == TFFR_OK) s = upload(P->kx, kxv);
  if (s == TFFR_OK) s = upload(P->ku, kuv);
  P->from_xy = kx_tab != nullptr;
  P->hku = kuv;
  {
    // Stolt baseline parts: the widest gap between consecutive samples in lattice units.
    // On the Stolt map the gap at sample p grows with |ku| (d kx / dk = 4k / kx), so the
    // slice of largest |ku| holds it.
    const double lscale = p->fov_x / (2.0 * kPi);
    double spmax = 0.0;
    auto row_gaps = [&](int n) {
      double prev = 0.0;
      for (int i = 0; i < p->n_freq; ++i) {
        const double kx = kx_tab ? kx_tab[(size_t)n * p->n_freq + i] : std::sqrt(4.0 * k[i] * k[i] - ku[n] * ku[n]);
        if (i > 0) spmax = std::max(spmax, (kx - prev) * lscale);
        prev = kx;
      }
    };
    if (kx_tab) {
      for (int n = 0; n < p->n_pulses; ++n) row_gaps(n);
    } else {
      int nmax = 0;
      for (int n = 1; n < p->n_pulses; ++n)
        if (std::fabs(ku[n]) > std::fabs(ku[nmax])) nmax = n;
      row_gaps(nmax);
    }
    P->stolt_part =
        spmax > 0.0 ? (int)std::max(1.0, std::min<double>(p->n_freq, std::floor((p->mx - 2) / spmax))) : p->n_freq;
  }
  if (s == TFFR_OK) s = upload(P->ystart, ys);
  if (s == TFFR_OK) s = upload(P->ycn, cn);
  if (s != TFFR_OK) return fail(s);

  // tFFR weight polynomial (float path, integer q only: the tap set is then constant on (0, 1))
  g.use_poly = 0;
  g.nseg = tffr::kPolySeg;
  g.deg = tffr::kPolyDeg;
  if (!P->dbl() && p->weighting == TFFR_W_TFFR && std::fabs(p->q - std::round(p->q)) < 1e-12) {
    std::vector<float> poly;
    if (fit_weight_poly(p->window_a, p->q, g.nseg, g.deg, poly)) {
      s = upload(P->poly, poly);
      if (s != TFFR_OK) return fail(s);
      g.use_poly = 1;
    }
  }

  // workspace layout
  size_t off = 0;
  P->off_hx = off;
  off = align_up(off + (size_t)p->n_pulses * p->mx * csz);
  P->off_h12 = off;  // entropy step: the two gradient fields, interleaved [n_pulses][mx][2]
  off = align_up(off + 2 * (size_t)p->n_pulses * p->mx * csz);
  P->off_cblk = off;  // entropy step: centring constant per column block
  off = align_up(off + (P->dbl() ? sizeof(double) : sizeof(float)) * (size_t)((p->mx + P->cb - 1) / P->cb));
  P->off_part = off;
  off = align_up(off + sizeof(double) * 2 * std::max<size_t>(kEntropyParts, (p->mx + P->cb - 1) / P->cb));
  P->off_stats = off;
  off = align_up(off + sizeof(double) * 2);
  P->step_bytes = off;  // the entropy step uses the regions above, nothing below
  P->off_kept = off;
  off = align_up(off + sizeof(unsigned long long) * kPartials);
  P->off_count = off;
  off = align_up(off + sizeof(long long));
  P->off_status = off;
  off = align_up(off + sizeof(int));
  if (p->weighting == TFFR_W_FFR) {
    s = ffr_route(p, hkx, &P->ffr_route, &P->ffr_halfband, &P->ffr_lmax);
    if (s != TFFR_OK) return fail(s);
    // route 0: the selected inversion yields the inverse on the band it factors; B_r may
    // reach beyond the frame product's own half-band, so factor with the wider of the two
    g.band_b = P->ffr_route == 0 ? std::max(P->ffr_halfband, p->band_r) : kFfrNormalBand;
    const size_t KT = 2 * ((size_t)std::ceil(p->q) + 1) + 1;
    if (P->ffr_route == 0 && (size_t)p->n_freq * (KT * sizeof(double) + sizeof(int)) > lds_max)
      return fail(TFFR_ERR_UNSUPPORTED);
    P->ffr_nwg = std::min(p->n_pulses, P->ffr_route == 0 ? 1024 : 512);
    P->off_gband = off;  // FFR scratch: per-workgroup bands, Gram matrices and reduction blocks
    off = align_up(off + tffr::ffr_scratch_bytes(g, P->ffr_route, P->ffr_lmax, P->ffr_nwg));
  }
  P->work_bytes = off;

  // plain FFR: solve once per geometry, keep D, report a singular frame product
  if (p->weighting == TFFR_W_FFR) {
    const size_t dbytes = (size_t)p->n_pulses * p->n_freq * (2 * p->band_r + 1) * P->rsize();
    void* work = nullptr;
    if (hipMalloc(&P->ffr_d.p, dbytes) != hipSuccess) return fail(TFFR_ERR_NOMEM);
    if (hipMalloc(&work, P->work_bytes) != hipSuccess) return fail(TFFR_ERR_NOMEM);
    char* wb = (char*)work;
    hipError_t e = hipMemset(wb + P->off_status, 0, sizeof(int));
    if (e == hipSuccess) {
      if (P->dbl())
        e = tffr::launch_ffr<double>(g, tables<double>(P), P->ffr_route, P->ffr_lmax, P->ffr_nwg,
                                     (double*)(wb + P->off_gband), (double*)P->ffr_d.p, (int*)(wb + P->off_status), 0);
      else
        e = tffr::launch_ffr<float>(g, tables<float>(P), P->ffr_route, P->ffr_lmax, P->ffr_nwg,
                                    (double*)(wb + P->off_gband), (float*)P->ffr_d.p, (int*)(wb + P->off_status), 0);
    }
    int st = 0;
    if (e == hipSuccess) e = hipMemcpy(&st, wb + P->off_status, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(work);
    if (e != hipSuccess) return fail(TFFR_ERR_HIP);
    P->ffr_status = st;
    const char* keep = std::getenv("TFFR_FFR_KEEP_SINGULAR");  // diagnostics: keep the plan, query the status
    if (st != 0 && !(keep && std::atoi(keep) == 1)) return fail(st == 2 ? TFFR_ERR_LAYOUT : TFFR_ERR_SINGULAR);
  }
  if (hipDeviceSynchronize() != hipSuccess) return fail(TFFR_ERR_HIP);
  P->scratch = scratch_for_device(P->device);  // device current: the plan's
  *out = P;
  return TFFR_OK;
}

}  // namespace

extern "C" {

tffr_status tffr_plan_create(const tffr_params* p, const double* k, const double* ku, tffr_plan** out) {
  if (!out) return TFFR_ERR_ARG;
  *out = nullptr;
  const tffr_status s = tffr_validate(p, k, ku);
  if (s != TFFR_OK) return s;
  return plan_create(p, k, ku, nullptr, out);
}

tffr_status tffr_plan_create_xy(const tffr_params* p, const double* kx, const double* ky, tffr_plan** out) {
  if (!out) return TFFR_ERR_ARG;
  *out = nullptr;
  const tffr_status s = tffr_validate_xy(p, kx, ky);
  if (s != TFFR_OK) return s;
  std::vector<double> ky_row(p->n_pulses);
  for (int n = 0; n < p->n_pulses; ++n) ky_row[n] = ky[(size_t)n * p->n_freq];
  return plan_create(p, nullptr, ky_row.data(), kx, out);
}

void tffr_plan_destroy(tffr_plan* plan) { delete plan; }

size_t tffr_workspace_bytes(const tffr_plan* plan) { return plan ? plan->work_bytes : 0; }

tffr_status tffr_plan_info(const tffr_plan* plan, int32_t* nfx, int32_t* nfy, double* beta, int32_t* hb) {
  if (!plan) return TFFR_ERR_ARG;
  if (nfx) *nfx = plan->geo.nfx;
  if (nfy) *nfy = plan->geo.nfy;
  if (beta) *beta = plan->beta;
  if (hb) *hb = plan->ffr_halfband;
  return TFFR_OK;
}


tffr_status tffr_forward(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw, void* img,
                         void* work, tffr_stream stream) {
  if (!P || !smp || !img || !work) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (!aligned(work, 16) || !aligned(img, P->csize() / 2) || !aligned(smp, 4)) return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_forward<double>(P, smp, ph, da, uw, img, work, st, -1)
                  : do_forward<float>(P, smp, ph, da, uw, img, work, st, -1);
}

tffr_status tffr_rma_front_end(tffr_plan* P, const void* echoes, int32_t n_positions, double du, double xc,
                               void* samples, tffr_stream stream) {
  if (!P || !echoes || !samples) return TFFR_ERR_ARG;
  if (P->from_xy || !(du > 0.0) || !std::isfinite(du) || !std::isfinite(xc)) return TFFR_ERR_ARG;
  const int J = n_positions, NU = P->prm.n_pulses;
  if (J < NU || J < 64 || (J & (J - 1)) != 0) return TFFR_ERR_ARG;
  if (J > 16384 || (P->dbl() && J > 8192)) return TFFR_ERR_UNSUPPORTED;
  // the plan's azimuth wavenumbers must be those of the J-point transform
  const double dku = 2.0 * kPi / ((double)J * du);
  for (int n = 0; n < NU; ++n)
    if (std::fabs(P->hku[n] - (n - NU / 2) * dku) > 1e-9 * dku * std::max(1, NU)) return TFFR_ERR_ARG;
  if (!aligned(echoes, P->csize() / 2) || !aligned(samples, 4)) return TFFR_ERR_LAYOUT;
  int logj = 0;
  while ((1 << logj) < J) ++logj;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e =
      P->dbl() ? tffr::launch_rma_front<double>(P->geo, tables<double>(P), logj, (const cplx<double>*)echoes, xc,
                                                sample_type(P), samples, st)
               : tffr::launch_rma_front<float>(P->geo, tables<float>(P), logj, (const cplx<float>*)echoes, xc,
                                               sample_type(P), samples, st);
  return hip_status(e);
}

tffr_status tffr_rma_range_fft(tffr_plan* P, const void* pulses, int32_t n_positions, const void* ref, void* echoes,
                               tffr_stream stream) {
  if (!P || !pulses || !echoes || n_positions < 1) return TFFR_ERR_ARG;
  const int Pf = P->prm.n_freq;
  if ((Pf & (Pf - 1)) != 0 || Pf < 64 || Pf > 16384 || (P->dbl() && Pf > 8192)) return TFFR_ERR_UNSUPPORTED;
  if (!aligned(pulses, P->csize() / 2) || !aligned(echoes, P->csize() / 2) || (ref && !aligned(ref, P->csize() / 2)))
    return TFFR_ERR_LAYOUT;
  int logp = 0;
  while ((1 << logp) < Pf) ++logp;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e =
      P->dbl() ? tffr::launch_rma_range_fft<double>(logp, n_positions, (const cplx<double>*)pulses,
                                                    (const cplx<double>*)ref, (cplx<double>*)echoes, st)
               : tffr::launch_rma_range_fft<float>(logp, n_positions, (const cplx<float>*)pulses,
                                                   (const cplx<float>*)ref, (cplx<float>*)echoes, st);
  return hip_status(e);
}

tffr_status tffr_rma_front_end_pos(tffr_plan* P, const void* echoes, int32_t n_positions, double du,
                                   const double* dpos, double xc, void* samples, tffr_stream stream) {
  if (!P || !echoes || !dpos || !samples) return TFFR_ERR_ARG;
  if (P->from_xy || !(du > 0.0) || !std::isfinite(du) || !std::isfinite(xc)) return TFFR_ERR_ARG;
  const int J = n_positions, NU = P->prm.n_pulses;
  if (J < NU || J < 64 || (J & (J - 1)) != 0) return TFFR_ERR_ARG;
  const double dku = 2.0 * kPi / ((double)J * du);
  for (int n = 0; n < NU; ++n)
    if (std::fabs(P->hku[n] - (n - NU / 2) * dku) > 1e-9 * dku * std::max(1, NU)) return TFFR_ERR_ARG;
  if (!aligned(echoes, P->csize() / 2) || !aligned(samples, 4)) return TFFR_ERR_LAYOUT;
  const int G = 1 << P->logfg, W = P->prm.kernel_width;
  if ((size_t)G * P->csize() + ((size_t)G / 64 + 64) * P->csize() > ((size_t)128 << 10) + 8192)
    return TFFR_ERR_UNSUPPORTED;
  // true positions on the periodic grid: g_j = G ((j - J/2) du + d_j) / (J du); strictly
  // increasing within one period, else TFFR_ERR_NONMONOTONE
  std::vector<double> gp(J);
  for (int j = 0; j < J; ++j) {
    if (!std::isfinite(dpos[j])) return TFFR_ERR_ARG;
    gp[j] = (double)G * (((double)j - J / 2.0) * du + dpos[j]) / ((double)J * du);
  }
  double gmin = gp[0] + G - gp[J - 1];  // the gap across the period
  for (int j = 1; j < J; ++j) gmin = std::min(gmin, gp[j] - gp[j - 1]);
  if (!(gmin > 0.0)) return TFFR_ERR_NONMONOTONE;
  // sub-passes: a power of two (dividing J) with S gmin > W + 1, so sources S apart, also
  // across the period, keep their taps apart; at most J (one source per sub-pass)
  int S = 1;
  while (S < J && S * gmin <= W + 1.0) S *= 2;
  hipStream_t st = (hipStream_t)stream;
  // the positions replace those of an earlier call only once its launch has finished
  if (hipStreamSynchronize(st) != hipSuccess) return TFFR_ERR_HIP;
  if (P->fpos_n < (size_t)J) {
    if (P->fpos.p) (void)hipFree(P->fpos.p);
    P->fpos.p = nullptr;
    P->fpos_n = 0;
    if (hipMalloc(&P->fpos.p, sizeof(double) * J) != hipSuccess) return TFFR_ERR_NOMEM;
    P->fpos_n = J;
  }
  if (hipMemcpy(P->fpos.p, gp.data(), sizeof(double) * J, hipMemcpyHostToDevice) != hipSuccess) return TFFR_ERR_HIP;
  const hipError_t e =
      P->dbl() ? tffr::launch_rma_front_pos<double>(P->geo, tables<double>(P), P->logfg, (const cplx<double>*)echoes,
                                                    (const double*)P->fpos.p, J, S, xc, sample_type(P), samples, st)
               : tffr::launch_rma_front_pos<float>(P->geo, tables<float>(P), P->logfg, (const cplx<float>*)echoes,
                                                   (const double*)P->fpos.p, J, S, xc, sample_type(P), samples, st);
  return hip_status(e);
}

tffr_status tffr_stolt_image(tffr_plan* P, const void* smp, const void* ph, const void* da, void* img, void* work,
                             tffr_stream stream) {
  if (!P || !smp || !img || !work) return TFFR_ERR_ARG;
  const int mx = P->prm.mx;
  if ((mx & (mx - 1)) != 0 || ((1 << P->geo.lognfx) % mx) != 0) return TFFR_ERR_UNSUPPORTED;
  if (!aligned(work, 16) || !aligned(img, P->csize() / 2) || !aligned(smp, 4)) return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_stolt<double>(P, smp, ph, da, img, work, st) : do_stolt<float>(P, smp, ph, da, img, work, st);
}

tffr_status tffr_adjoint(tffr_plan* P, const void* cot, const void* smp, const void* ph, const void* da, const void* uw,
                         void* gs, void* gph, void* gda, void* work, tffr_stream stream) {
  if (!P || !cot || !gs || !work) return TFFR_ERR_ARG;
  if ((gph || gda) && !smp) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (!aligned(work, 16) || !aligned(cot, P->csize() / 2) || !aligned(gs, P->csize() / 2)) return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_adjoint<double>(P, cot, smp, ph, da, uw, gs, gph, gda, work, st)
                  : do_adjoint<float>(P, cot, smp, ph, da, uw, gs, gph, gda, work, st);
}

tffr_status tffr_entropy(tffr_plan* P, const void* img, double* loss, void* grad, void* work, tffr_stream stream) {
  if (!P || !img || !loss || !work) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  double* part = (double*)((char*)work + P->off_part);
  const size_t count = (size_t)P->prm.mx * P->prm.my;
  const int nparts = (int)std::max<size_t>(1, std::min<size_t>(kEntropyParts, (count + 1023) / 1024));
  hipError_t e = P->dbl() ? tffr::launch_entropy<double>(P->geo, (const cplx<double>*)img, part, nparts, loss,
                                                         (cplx<double>*)grad, st)
                          : tffr::launch_entropy<float>(P->geo, (const cplx<float>*)img, part, nparts, loss,
                                                        (cplx<float>*)grad, st);
  return hip_status(e);
}

tffr_status tffr_entropy_step(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw, void* img,
                              double* loss, void* gs, void* gph, void* gda, void* work, tffr_stream stream) {
  if (!P || !smp || !img || !loss || !gs || !work) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (!aligned(work, 16) || !aligned(img, P->csize() / 2) || !aligned(gs, P->csize() / 2)) return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_entropy_step<double>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st)
                  : do_entropy_step<float>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st);
}

tffr_status tffr_entropy_step_noalloc(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw,
                                      void* img, double* loss, void* gs, void* gph, void* gda, tffr_stream stream) {
  if (!P || !smp || !img || !loss || !gs) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (P->step_bytes > (size_t)TFFR_SCRATCH_BYTES) return TFFR_ERR_SCRATCH;
  if (!P->scratch) return TFFR_ERR_HIP;
  if (!aligned(img, P->csize() / 2) || !aligned(gs, P->csize() / 2)) return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_entropy_step<double>(P, smp, ph, da, uw, img, loss, gs, gph, gda, P->scratch, st)
                  : do_entropy_step<float>(P, smp, ph, da, uw, img, loss, gs, gph, gda, P->scratch, st);
}

tffr_status tffr_coord_grad(tffr_plan* P, const void* cot, const void* smp, const void* ph, const void* da,
                            const void* uw, void* gkx, void* gky, void* work, tffr_stream stream) {
  if (!P || !cot || !smp || !gkx || !gky || !work) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (!aligned(work, 16) || !aligned(cot, P->csize() / 2) || !aligned(smp, 4) || !aligned(gkx, P->rsize()) ||
      !aligned(gky, P->rsize()))
    return TFFR_ERR_LAYOUT;
  if (!P->coord_cb) return TFFR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)work;
  hipError_t e;
  if (P->dbl()) {
    const double* w = (const double*)uw;
    if (!w && P->prm.weighting == TFFR_W_FFR) w = (const double*)P->ffr_d.p;
    e = tffr::launch_coord_grad<double>(P->geo, tables<double>(P), P->coord_cb, sample_type(P),
                                        (const cplx<double>*)cot, smp, (const double*)ph, (const double*)da, w,
                                        (cplx<double>*)(wb + P->off_hx), (cplx<double>*)(wb + P->off_h12),
                                        (double*)gkx, (double*)gky, st);
  } else {
    const float* w = (const float*)uw;
    if (!w && P->prm.weighting == TFFR_W_FFR) w = (const float*)P->ffr_d.p;
    e = tffr::launch_coord_grad<float>(P->geo, tables<float>(P), P->coord_cb, sample_type(P),
                                       (const cplx<float>*)cot, smp, (const float*)ph, (const float*)da, w,
                                       (cplx<float>*)(wb + P->off_hx), (cplx<float>*)(wb + P->off_h12),
                                       (float*)gkx, (float*)gky, st);
  }
  return hip_status(e);
}

tffr_status tffr_row_phase_grad(tffr_plan* P, const void* smp, const void* gs, void* gph, void* gda,
                                tffr_stream stream) {
  if (!P || !smp || !gs || !gph) return TFFR_ERR_ARG;
  if (!aligned(gs, P->csize() / 2) || !aligned(smp, 4) || !aligned(gph, P->rsize()) ||
      (gda && !aligned(gda, P->rsize())))
    return TFFR_ERR_LAYOUT;
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e =
      P->dbl() ? tffr::launch_row_phase_grad<double>(P->geo, tables<double>(P), sample_type(P), smp,
                                                     (const cplx<double>*)gs, (double*)gph, (double*)gda, st)
               : tffr::launch_row_phase_grad<float>(P->geo, tables<float>(P), sample_type(P), smp,
                                                    (const cplx<float>*)gs, (float*)gph, (float*)gda, st);
  return hip_status(e);
}

tffr_status tffr_weights(tffr_plan* P, void* d_w, void* work, tffr_stream stream) {
  if (!P || !d_w || !work) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)work;
  hipError_t e;
  if (P->prm.weighting == TFFR_W_FFR) {
    int* status = (int*)(wb + P->off_status);
    e = P->dbl() ? tffr::launch_ffr<double>(P->geo, tables<double>(P), P->ffr_route, P->ffr_lmax, P->ffr_nwg,
                                            (double*)(wb + P->off_gband), (double*)d_w, status, st)
                 : tffr::launch_ffr<float>(P->geo, tables<float>(P), P->ffr_route, P->ffr_lmax, P->ffr_nwg,
                                           (double*)(wb + P->off_gband), (float*)d_w, status, st);
  } else {
    unsigned long long* kept = (unsigned long long*)(wb + P->off_kept);
    e = P->dbl() ? tffr::launch_weights<double>(P->geo, tables<double>(P), (double*)d_w, kept, kPartials, st)
                 : tffr::launch_weights<float>(P->geo, tables<float>(P), (float*)d_w, kept, kPartials, st);
  }
  return hip_status(e);
}

tffr_status tffr_kept_count(tffr_plan* P, void* work, int64_t* count, tffr_stream stream) {
  if (!P || !work || !count) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)work;
  unsigned long long* kept = (unsigned long long*)(wb + P->off_kept);
  long long* dcount = (long long*)(wb + P->off_count);
  hipError_t e = P->dbl() ? tffr::launch_weights<double>(P->geo, tables<double>(P), nullptr, kept, kPartials, st)
                          : tffr::launch_weights<float>(P->geo, tables<float>(P), nullptr, kept, kPartials, st);
  if (e == hipSuccess) e = tffr::launch_sum_u64(kept, kPartials, dcount, st);
  long long h = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&h, dcount, sizeof(h), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return TFFR_ERR_HIP;
  *count = (int64_t)h;
  return TFFR_OK;
}

tffr_status tffr_debug_fft(int32_t log2n, int32_t batch, int32_t sign, int32_t max_radix, int32_t dtype,
                           const void* in, void* out, tffr_stream stream) {
  if (log2n < 6 || log2n > kMaxLogN || batch < 1 || (sign != 1 && sign != -1) || !in || !out) return TFFR_ERR_ARG;
  if (max_radix != 8 && max_radix != 16) return TFFR_ERR_ARG;
  if (dtype != TFFR_C64 && dtype != TFFR_C128) return TFFR_ERR_UNSUPPORTED;
  const size_t csz = dtype == TFFR_C128 ? 16 : 8;
  if (csz * (((size_t)1 << log2n) + ((size_t)1 << log2n) / 64 + 64) > tffr::max_dynamic_lds())
    return TFFR_ERR_UNSUPPORTED;
  const int n = 1 << log2n;
  hipStream_t st = (hipStream_t)stream;
  std::vector<double> tw = twiddle_table(n);
  DevBuf dtw;
  tffr_status s = dtype == TFFR_C128 ? upload(dtw, tw) : upload(dtw, cast<float>(tw));
  if (s != TFFR_OK) return s;
  hipError_t e = dtype == TFFR_C128
                     ? tffr::launch_fft<double>(log2n, batch, sign, max_radix, (const cplx<double>*)in, (cplx<double>*)out,
                                                (const cplx<double>*)dtw.p, st)
                     : tffr::launch_fft<float>(log2n, batch, sign, max_radix, (const cplx<float>*)in, (cplx<float>*)out,
                                               (const cplx<float>*)dtw.p, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);  // the twiddle table is freed on return
  return hip_status(e);
}

tffr_status tffr_debug_rows(tffr_plan* P, int32_t stage, const void* smp, const void* ph, const void* da,
                            const void* uw, void* out, tffr_stream stream) {
  if (!P || !smp || !out || (stage != 0 && stage != 1)) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  return P->dbl() ? do_forward<double>(P, smp, ph, da, uw, out, nullptr, st, stage)
                  : do_forward<float>(P, smp, ph, da, uw, out, nullptr, st, stage);
}

tffr_status tffr_debug_cols(tffr_plan* P, const void* hx, void* img, tffr_stream stream) {
  if (!P || !hx || !img) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = P->dbl() ? tffr::launch_fwd_cols<double>(P->geo, tables<double>(P), P->cb, (const cplx<double>*)hx,
                                                          (cplx<double>*)img, nullptr, st)
                          : tffr::launch_fwd_cols<float>(P->geo, tables<float>(P), P->cb, (const cplx<float>*)hx,
                                                         (cplx<float>*)img, nullptr, st);
  return hip_status(e);
}

tffr_status tffr_debug_ent_adj_rows(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw,
                                    double* loss, void* gs, void* gph, void* gda, void* work, tffr_stream stream) {
  if (!P || !smp || !loss || !gs || !work) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  if (!P->ent_fused) return TFFR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e;
  if (P->dbl()) {
    const double* w = (const double*)uw;
    if (!w && P->prm.weighting == TFFR_W_FFR) w = (const double*)P->ffr_d.p;
    e = launch_ent_adj_rows<double>(P, smp, ph, da, w, loss, gs, gph, gda, work, st);
  } else {
    const float* w = (const float*)uw;
    if (!w && P->prm.weighting == TFFR_W_FFR) w = (const float*)P->ffr_d.p;
    e = launch_ent_adj_rows<float>(P, smp, ph, da, w, loss, gs, gph, gda, work, st);
  }
  return hip_status(e);
}

tffr_status tffr_debug_step_kernel_times(tffr_plan* P, const void* smp, const void* ph, const void* da, const void* uw,
                                         void* img, double* loss, void* gs, void* gph, void* gda, void* work,
                                         tffr_stream stream, int32_t nsteps, float* ms_out, int32_t* nkern,
                                         const char** names) {
  if (!P || !smp || !img || !loss || !gs || !work || !ms_out || !nkern || nsteps < 1) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  EventMarks m{};
  m.st = st;
  int created = 0;
  hipError_t e = hipSuccess;
  for (; created < 8 && e == hipSuccess; ++created) e = hipEventCreate(&m.ev[created]);
  if (e != hipSuccess) --created;
  std::vector<double> acc(7, 0.0);
  int nk = 0;
  tffr_status s = e == hipSuccess ? TFFR_OK : TFFR_ERR_HIP;
  for (int it = 0; it < nsteps && s == TFFR_OK; ++it) {
    s = P->dbl() ? do_entropy_step<double>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st, record_mark, &m, &nk)
                 : do_entropy_step<float>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st, record_mark, &m, &nk);
    if (s == TFFR_OK && hipEventSynchronize(m.ev[nk]) != hipSuccess) s = TFFR_ERR_HIP;
    for (int i = 0; i < nk && s == TFFR_OK; ++i) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, m.ev[i], m.ev[i + 1]) != hipSuccess) s = TFFR_ERR_HIP;
      acc[i] += ms;
    }
  }
  for (int i = 0; i < created; ++i) (void)hipEventDestroy(m.ev[i]);
  if (s != TFFR_OK) return s;
  for (int i = 0; i < nk; ++i) ms_out[i] = (float)(acc[i] / nsteps);
  *nkern = nk;
  if (names) step_kernel_names(P, names);
  return TFFR_OK;
}

tffr_status tffr_debug_step_kernel_marginal_times(tffr_plan* P, const void* smp, const void* ph, const void* da,
                                                  const void* uw, void* img, double* loss, void* gs, void* gph,
                                                  void* gda, void* work, tffr_stream stream, int32_t nsteps,
                                                  float* ms_out, int32_t* nkern, const char** names) {
  if (!P || !smp || !img || !loss || !gs || !work || !ms_out || !nkern || nsteps < 1) return TFFR_ERR_ARG;
  if (P->prm.weighting == TFFR_W_USER && !uw) return TFFR_ERR_ARG;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t ev[2];
  if (hipEventCreate(&ev[0]) != hipSuccess) return TFFR_ERR_HIP;
  if (hipEventCreate(&ev[1]) != hipSuccess) {
    (void)hipEventDestroy(ev[0]);
    return TFFR_ERR_HIP;
  }
  // nsteps steps with launch `dup` issued twice (dup = -1: the plain step), events only
  // around the loop, after one untimed step of the same kind
  int nk = 0;
  auto loop_ms = [&](int dup, double* ms) -> tffr_status {
    tffr_status s = TFFR_OK;
    for (int it = -1; it < nsteps && s == TFFR_OK; ++it) {
      if (it == 0 && hipEventRecord(ev[0], st) != hipSuccess) return TFFR_ERR_HIP;
      s = P->dbl() ? do_entropy_step<double>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st, nullptr, nullptr,
                                             &nk, dup)
                   : do_entropy_step<float>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st, nullptr, nullptr,
                                            &nk, dup);
    }
    if (s != TFFR_OK) return s;
    float t = 0.0f;
    if (hipEventRecord(ev[1], st) != hipSuccess || hipEventSynchronize(ev[1]) != hipSuccess ||
        hipEventElapsedTime(&t, ev[0], ev[1]) != hipSuccess)
      return TFFR_ERR_HIP;
    *ms = (double)t / nsteps;
    return TFFR_OK;
  };
  double base = 0.0, with = 0.0;
  tffr_status s = loop_ms(-1, &base);
  const int n = nk;
  for (int i = 0; i < n && s == TFFR_OK; ++i) {
    s = loop_ms(i, &with);
    if (s == TFFR_OK) ms_out[i] = (float)(with - base);
  }
  if (s == TFFR_OK) {  // one plain step: the outputs are those of one step
    s = P->dbl() ? do_entropy_step<double>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st)
                 : do_entropy_step<float>(P, smp, ph, da, uw, img, loss, gs, gph, gda, work, st);
    if (s == TFFR_OK && hipStreamSynchronize(st) != hipSuccess) s = TFFR_ERR_HIP;
  }
  (void)hipEventDestroy(ev[0]);
  (void)hipEventDestroy(ev[1]);
  if (s != TFFR_OK) return s;
  *nkern = n;
  if (names) step_kernel_names(P, names);
  return TFFR_OK;
}

tffr_status tffr_debug_ffr_route(const tffr_plan* P, int32_t* route, int32_t* lattice_max, int32_t* solve_status) {
  if (!P) return TFFR_ERR_ARG;
  if (P->prm.weighting != TFFR_W_FFR) return TFFR_ERR_ARG;
  if (route) *route = P->ffr_route;
  if (lattice_max) *lattice_max = P->ffr_lmax;
  if (solve_status) *solve_status = P->ffr_status;
  return TFFR_OK;
}

tffr_status tffr_debug_plan_config(const tffr_plan* P, int32_t* range_mode, int32_t* az_cols, int32_t* ent_fused) {
  if (!P) return TFFR_ERR_ARG;
  if (range_mode) {
    *range_mode = P->geo.range_mode;
    if (P->geo.range_mode == 1 && P->geo.run_pair) *range_mode = 2;
    else if (P->geo.range_mode == 1 && P->geo.run_parts == 2) *range_mode = 3;
  }
  if (az_cols) *az_cols = P->cb;
  if (ent_fused) *ent_fused = P->ent_fused ? 1 : 0;
  return TFFR_OK;
}

tffr_status tffr_debug_ent_cols(tffr_plan* P, const void* hx, void* img, void* h12, void* work, tffr_stream stream) {
  if (!P || !hx || !img || !h12 || !work) return TFFR_ERR_ARG;
  if (!P->ent_fused) return TFFR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  char* wb = (char*)work;
  double* part = (double*)(wb + P->off_part);
  hipError_t e =
      P->dbl() ? tffr::launch_ent_cols<double>(P->geo, tables<double>(P), P->cb, (const cplx<double>*)hx,
                                               (cplx<double>*)img, part, (double*)(wb + P->off_cblk),
                                               (cplx<double>*)h12, st)
               : tffr::launch_ent_cols<float>(P->geo, tables<float>(P), P->cb, (const cplx<float>*)hx,
                                              (cplx<float>*)img, part, (float*)(wb + P->off_cblk),
                                              (cplx<float>*)h12, st);
  return hip_status(e);
}

}  // extern "C"
