// HIP kernels of libtffr for gfx950 (CDNA4).
//
// The image I[jx,jy] = sum_{n,p} c[n,p] exp(i (kx[n,p] X[jx] + ky[n] Y[jy])) separates
// along the slice structure of stripmap data (each azimuth slice n has one ky, its
// samples are non-uniform in kx only; Sec. II-A and Algorithm 1):
//
//   range stage    Hx[n][jx] = sum_p c[n,p] exp(i kx[n,p] X[jx])         one slice per workgroup
//   azimuth stage  I[jx][jy] = sum_n Hx[n][jx] exp(i ky[n] Y[jy])        CB range columns per workgroup
//
// Each stage is a 1-D type-1 NUFFT done entirely in LDS: spread with an
// exponential-of-semicircle (ES) kernel onto an oversampled periodic grid, Stockham
// radix-16 FFT, keep the centred bins and divide by the kernel's transform.  The
// adjoint runs the two type-2 stages in reverse.  Samples are read once, each
// intermediate is written once and read once, and nothing is done with global atomics.
//
// Coordinates are reduced in FP64 (kx up to ~430 rad/m times pixel sizes makes
// phases of ~1e4 rad) and kept as an (integer cell, FP32 fraction) pair.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "tffr_internal.h"

namespace tffr {

#define TFFR_PI 3.141592653589793

// ----------------------------------------------------------------------------- complex
template <typename R>
__device__ __forceinline__ cplx<R> operator+(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> operator-(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> operator*(R s, cplx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cplx<R> cmulc(cplx<R> a, cplx<R> b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <int SIGN, typename R>
__device__ __forceinline__ cplx<R> mul_si(cplx<R> a) {  // a * (SIGN i)
  return SIGN > 0 ? cplx<R>{-a.y, a.x} : cplx<R>{a.y, -a.x};
}

// ----------------------------------------------------------------------------- launch mapping
// Workgroups are dealt to the 8 XCDs round-robin (blockIdx mod 8).  Renumber them so the
// workgroups one XCD runs get consecutive logical indices: neighbouring column blocks,
// which share cache lines of the range-spectra array, then meet in the same L2.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
  constexpr int NX = 8;
  const int xcd = bid % NX, local = bid / NX, base = nblocks / NX, rem = nblocks % NX;
  return xcd * base + min(xcd, rem) + local;
}

// ----------------------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

template <int NT>
__device__ double block_sum(double v) {
  __shared__ double red[NT / 64];
  v = wave_sum(v);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t += red[i];
  return t;
}

// ----------------------------------------------------------------------------- LDS FFT
// Small DFTs in registers: X[k] = sum_r x[r] exp(SIGN 2 pi i r k / R).
template <int SIGN, typename R>
__device__ __forceinline__ void dft2(cplx<R>* a) {
  cplx<R> t = a[0];
  a[0] = t + a[1];
  a[1] = t - a[1];
}
template <int SIGN, typename R>
__device__ __forceinline__ void dft4(cplx<R>* a) {
  cplx<R> s0 = a[0] + a[2], d0 = a[0] - a[2];
  cplx<R> s1 = a[1] + a[3], d1 = mul_si<SIGN>(a[1] - a[3]);
  a[0] = s0 + s1;
  a[2] = s0 - s1;
  a[1] = d0 + d1;
  a[3] = d0 - d1;
}
template <int SIGN, typename R>
__device__ __forceinline__ void dft8(cplx<R>* a) {
  cplx<R> e[4] = {a[0], a[2], a[4], a[6]};
  cplx<R> o[4] = {a[1], a[3], a[5], a[7]};
  dft4<SIGN>(e);
  dft4<SIGN>(o);
  const R h = R(0.70710678118654752440);
  // twiddles exp(SIGN 2 pi i k / 8): (1 + SIGN i)/sqrt2, SIGN i, (-1 + SIGN i)/sqrt2
  cplx<R> o1 = {h * (o[1].x - R(SIGN) * o[1].y), h * (o[1].y + R(SIGN) * o[1].x)};
  cplx<R> o2 = mul_si<SIGN>(o[2]);
  cplx<R> o3 = {h * (-o[3].x - R(SIGN) * o[3].y), h * (-o[3].y + R(SIGN) * o[3].x)};
  a[0] = e[0] + o[0];
  a[4] = e[0] - o[0];
  a[1] = e[1] + o1;
  a[5] = e[1] - o1;
  a[2] = e[2] + o2;
  a[6] = e[2] - o2;
  a[3] = e[3] + o3;
  a[7] = e[3] - o3;
}
// 16-point DFT as 4 x 4: four 4-point DFTs over r = r1 + 4 r2 (stride 4), twiddles
// exp(SIGN 2 pi i r1 k2 / 16), four 4-point DFTs over r1; output index k2 + 4 k1.
template <int SIGN, typename R>
__device__ __forceinline__ void dft16(cplx<R>* a) {
  cplx<R> t[16];
#pragma unroll
  for (int r1 = 0; r1 < 4; ++r1) {
    cplx<R> u[4] = {a[r1], a[r1 + 4], a[r1 + 8], a[r1 + 12]};
    dft4<SIGN>(u);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[r1 * 4 + k2] = u[k2];
  }
  const R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), h = R(0.70710678118654752440);
  // exp(SIGN 2 pi i m / 16) for m = r1 k2 in {1, 2, 3, 4, 6, 9}
  auto rot = [&](cplx<R> v, int m) -> cplx<R> {
    R cr, ci;
    switch (m) {
      case 1: cr = c1; ci = s1; break;
      case 2: cr = h; ci = h; break;
      case 3: cr = s1; ci = c1; break;
      case 4: cr = 0; ci = 1; break;
      case 6: cr = -h; ci = h; break;
      default: cr = -c1; ci = -s1; break;  // m = 9
    }
    ci = R(SIGN) * ci;
    return {v.x * cr - v.y * ci, v.x * ci + v.y * cr};
  };
#pragma unroll
  for (int r1 = 1; r1 < 4; ++r1)
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) t[r1 * 4 + k2] = rot(t[r1 * 4 + k2], r1 * k2);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cplx<R> u[4] = {t[k2], t[4 + k2], t[8 + k2], t[12 + k2]};
    dft4<SIGN>(u);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) a[k2 + 4 * k1] = u[k1];
  }
}

template <int SIGN, int RAD, typename R>
__device__ __forceinline__ void dft(cplx<R>* a) {
  if constexpr (RAD == 16) dft16<SIGN>(a);
  else if constexpr (RAD == 8) dft8<SIGN>(a);
  else if constexpr (RAD == 4) dft4<SIGN>(a);
  else dft2<SIGN>(a);
}

// Twiddle exp(+2 pi i m / N) from the two-level LDS table tw = [hi (N/64)] [lo (64)]:
// exp(2 pi i m / N) = hi[m / 64] * lo[m % 64].
template <int N, typename R>
__device__ __forceinline__ cplx<R> twiddle(const cplx<R>* tw, int m) {
  return cmul(tw[m >> 6], tw[N / 64 + (m & 63)]);
}
template <int N>
constexpr int tw_entries() {
  return N / 64 + 64;
}
// Copy the two-level twiddle table of length-N transforms into LDS (caller barriers).
template <int N, int NT, typename R>
__device__ __forceinline__ void load_twiddles(cplx<R>* tw, const cplx<R>* __restrict__ g) {
  for (int i = threadIdx.x; i < tw_entries<N>(); i += NT) tw[i] = g[i];
}

// LDS position of element j of a transform between two FFT stages (the range kernels'
// layout).  A stage's stores y[(i - k) RAD + k + r P] put consecutive lanes RAD apart
// when P = 1 (and in runs of P when P is small), so a plain layout sends many lanes of a
// store to the same bank.  The position XORs bits 0..4 of j with bits 5..8 (into bits
// 0..3) and 6..7 (into bits 3..4): a bijection that moves nothing across a 32-element
// block, so the loads x[i + r N/RAD] of consecutive lanes stay on distinct banks while
// the small-P stores spread out.  Transforms are still read from and written back to
// the natural layout; only the values between stages live in this one.  For a and b
// with no common bits the position of a + b is swz(a) ^ swz(b) (swz is linear over
// XOR): one swz per butterfly, then one XOR with a constant per element.
__host__ __device__ constexpr int swz(int j) { return j ^ ((j >> 5) & 15) ^ (((j >> 6) & 3) << 3); }

// One Stockham autosort stage of radix RAD after spans P, on NBAT transforms stored
// back to back (in place: all reads, barrier, all writes, barrier).  Butterfly i of a
// transform reads x[i + r N/RAD], applies exp(SIGN 2 pi i r k / (P RAD)) with
// k = i mod P, and writes y[(i - k) RAD + k + r P].  SWI / SWO: input / output in the
// inter-stage layout (swz).
template <int SIGN, int N, int RAD, int P, int NT, int NBAT, bool SWI, bool SWO, typename R>
__device__ __forceinline__ void fft_stage(cplx<R>* buf, const cplx<R>* tw) {
  constexpr int NB = N / RAD;
  constexpr int TOT = NB * NBAT;
  constexpr int BPT = (TOT + NT - 1) / NT;
  cplx<R> v[BPT][RAD];
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int bf = threadIdx.x + b * NT;
    if (TOT % NT == 0 || bf < TOT) {
      const int col = bf / NB, i = bf - col * NB;
      const cplx<R>* x = buf + col * N;
      const int si = swz(i);
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[b][r] = x[SWI ? (si ^ swz(r * NB)) : (i + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < BPT; ++b) {
    const int bf = threadIdx.x + b * NT;
    if (TOT % NT == 0 || bf < TOT) {
      const int col = bf / NB, i = bf - col * NB;
      const int k = i & (P - 1);
      if constexpr (P > 1) {
        // one table lookup w = exp(SIGN 2 pi i k / (P RAD)); the other powers by
        // short product chains (w^2 = w w, w^3 = w^2 w, w^4 = w^2 w^2, w^r = w^(r-4) w^4)
        constexpr int STEP = N / (P * RAD);
        cplx<R> wp[RAD];
        wp[1] = twiddle<N>(tw, k * STEP);
        if (SIGN < 0) wp[1].y = -wp[1].y;
        if constexpr (RAD >= 4) {
          wp[2] = cmul(wp[1], wp[1]);
          wp[3] = cmul(wp[2], wp[1]);
        }
        if constexpr (RAD >= 8) {
          wp[4] = cmul(wp[2], wp[2]);
          wp[5] = cmul(wp[4], wp[1]);
          wp[6] = cmul(wp[3], wp[3]);
          wp[7] = cmul(wp[4], wp[3]);
        }
        if constexpr (RAD == 16) {
#pragma unroll
          for (int r = 8; r < 16; ++r) wp[r] = cmul(wp[r - 4], wp[4]);
        }
#pragma unroll
        for (int r = 1; r < RAD; ++r) v[b][r] = cmul(v[b][r], wp[r]);
      }
      dft<SIGN, RAD>(v[b]);
      const int j = (i - k) * RAD + k;
      cplx<R>* y = buf + col * N;
      const int sj = swz(j);
#pragma unroll
      for (int r = 0; r < RAD; ++r) y[SWO ? (sj ^ swz(r * P)) : (j + r * P)] = v[b][r];
    }
  }
  __syncthreads();
}

template <int SIGN, int N, int P, int NT, int NBAT, int MAXRAD, int SWZ, typename R>
__device__ __forceinline__ void fft_from(cplx<R>* buf, const cplx<R>* tw) {
  if constexpr (P < N) {
    constexpr int RAD = (N / P) >= MAXRAD ? MAXRAD : (N / P);
    constexpr bool in = P > 1 && (SWZ == 1 || (SWZ == 2 && P == MAXRAD));
    constexpr bool out = P * RAD < N && (SWZ == 1 || (SWZ == 2 && P == 1));
    fft_stage<SIGN, N, RAD, P, NT, NBAT, in, out>(buf, tw);
    fft_from<SIGN, N, P * RAD, NT, NBAT, MAXRAD, SWZ>(buf, tw);
  }
}

// out[j] = sum_g buf[g] exp(SIGN 2 pi i g j / N) for NBAT transforms stored back to back
// in LDS, in place, natural order; tw is the LDS twiddle table.  Call with all NT
// threads after a barrier.
// Stages of radix MAXRAD (8 or 16) and one smaller last stage.  Radix 16 takes fewer LDS
// passes and, in the dense-slice range kernel, fewer registers (more workgroups per CU);
// radix 8 keeps more threads busy per stage where a workgroup has few butterflies.
// SWZ: 0 plain layout; 1 every value between stages in the bank-spreading layout
// (swz); 2 only the first stage's output (its stride-RAD stores conflict most).  Mode 1
// where a thread takes one butterfly per stage; with two (the entropy step's two-field
// adjoint transforms) the per-element addresses of mode 1 cost more registers than the
// conflicts cost time, mode 2 fits.
template <int SIGN, int N, int NT, int NBAT = 1, int MAXRAD = 8, int SWZ = 0, typename R>
__device__ __forceinline__ void lds_fft(cplx<R>* buf, const cplx<R>* tw) {
  fft_from<SIGN, N, 1, NT, NBAT, MAXRAD, SWZ>(buf, tw);
}

// ----------------------------------------------------------------------------- geometry
// Stolt map (FP64, no contraction) and lattice coordinate lam = kx fov_x / (2 pi),
// formed as (cycles per pixel) * mx.
__device__ __forceinline__ double stolt_kx(double k, double ku) {
#pragma clang fp contract(off)
  return sqrt(4.0 * (k * k) - ku * ku);
}
__device__ __forceinline__ double lattice_coord(double kx, const Geo& g) {
  return (kx * g.tx_scale) * (double)g.mx;
}
// Range wavenumber of sample (n, p) in two steps, so the load can be issued early: the
// raw value (k[p], or the explicit kx[n][p] of a plan made from coordinates), then kx.
template <typename R>
__device__ __forceinline__ double raw_k(const Tab<R>& t, int n_freq, int n, int p) {
  return t.kx ? t.kx[(size_t)n * n_freq + p] : t.k[p];
}
template <typename R>
__device__ __forceinline__ double kx_of(const Tab<R>& t, double raw, double ku) {
  return t.kx ? raw : stolt_kx(raw, ku);
}

// g(delta) = sum_{|k - delta| < q} R_Psi(k - delta) R_W(k - delta): the diagonal of the
// truncated frame product for a sample at fractional lattice offset delta.  R_W and R_Psi
// are the finite-interval cosine transforms of w = exp(-a|t|) and 1/w over [-1/2, 1/2]
// (the entries of W and Psi on the image's own lattice), with b = 2 pi d:
//   R_W(d) = 2 (a + e^{-a/2} (b sin(b/2) - a cos(b/2))) / (a^2 + b^2),
//   R_Psi(d) = 2 (e^{a/2} (b sin(b/2) + a cos(b/2)) - a) / (a^2 + b^2);
// ema2 = exp(-a/2), epa2 = exp(a/2).  Every tap
// has b/2 = pi (k - delta), so one sincos(pi delta) serves them all:
// sin(pi (k - delta)) = -(-1)^k sin(pi delta), cos(pi (k - delta)) = (-1)^k cos(pi delta).
__device__ double frame_diag(double delta, double a, double q, double ema2, double epa2) {
  const int K = (int)ceil(q) + 1;
  double sd, cd;
  sincospi(delta, &sd, &cd);
  double acc = 0.0;
  for (int k = -K; k <= K; ++k) {
    const double d = (double)k - delta;
    if (fabs(d) < q) {
      const double sg = (k & 1) ? -1.0 : 1.0;
      const double sn = -sg * sd, cs = sg * cd;
      const double b = 2.0 * TFFR_PI * d;
      const double den = a * a + b * b;
      const double rw = den == 0.0 ? 1.0 : 2.0 * (a + ema2 * (b * sn - a * cs)) / den;
      const double rp = den == 0.0 ? 1.0 : 2.0 * (epa2 * (b * sn + a * cs) - a) / den;
      acc += rp * rw;
    }
  }
  return acc;
}

// R_tau(1/g) in FP64 from the closed form (the double path, and float samples whose
// polynomial value falls within near_rel of the threshold).  Kept out of line (it is
// rarely taken and large); scalars by value so the caller keeps its state in registers.
__device__ __attribute__((noinline)) double tffr_weight_f64(double delta, double a, double q, double ema2,
                                                            double epa2, double tau, int mode) {
  const double gd = frame_diag(delta, a, q, ema2, epa2);
  const double inv = gd != 0.0 ? 1.0 / gd : 0.0;
  const bool keep = mode == 0 ? (fabs(inv) >= tau) : (gd >= tau);
  return keep ? inv : 0.0;
}

// tFFR weight R_tau(1/g) of a sample at lattice coordinate lam; poly is the piecewise
// polynomial of 1/g in the local variable of each segment, coefficient-major
// (poly[i * kPolySeg + seg]; LDS copy on the float path).
template <typename R>
__device__ __forceinline__ R tffr_weight(const Geo& g, const float* poly, double lam) {
  const double delta = lam - floor(lam);
  if (delta == 0.0) return g.keep0 ? (R)g.inv_g0 : (R)0;
  if (sizeof(R) == 4 && g.use_poly) {
    const double xs = delta * kPolySeg;
    const int seg = min((int)xs, kPolySeg - 1);
    const float t = (float)(2.0 * (xs - seg) - 1.0);
    const float* c = poly + seg;
    float v = c[0];
#pragma unroll
    for (int i = 1; i <= kPolyDeg; ++i) v = fmaf(v, t, c[i * kPolySeg]);
    const float thr = g.thr_f;
    if (fabsf(v - thr) > g.near_f * thr) {
      const bool keep = g.thresh_mode == 0 ? (v >= thr) : (v <= thr);
      return keep ? (R)v : (R)0;
    }
  }
  return (R)tffr_weight_f64(delta, g.a, g.q, g.ema2, g.epa2, g.tau, g.thresh_mode);
}

// Copy the tFFR weight polynomial into LDS (float path); returns the pointer to use.
template <int NT>
__device__ __forceinline__ const float* load_poly(const Geo& g, const float* __restrict__ gp, float* lp) {
  if (!gp) return gp;
  const int n = kPolySeg * (kPolyDeg + 1);
  for (int i = threadIdx.x; i < n; i += NT) lp[i] = gp[i];
  return lp;
}
constexpr int kPolyLds = 512;  // floats reserved in LDS for the weight polynomial

// Weight of sample (n, p) for the diagonal methods.
template <typename R>
__device__ __forceinline__ R diag_weight(const Geo& g, const Tab<R>& t, const float* poly, double ku, int n, int p,
                                         double lam) {
  switch (g.weighting) {
    case 3:  // tFFR
      return tffr_weight<R>(g, poly, lam);
    case 1: {  // trapezoid quadrature in lam along the slice
      if (g.n_freq == 1) return (R)1;
      const int plo = p > 0 ? p - 1 : 0, phi = p < g.n_freq - 1 ? p + 1 : g.n_freq - 1;
      const double llo = lattice_coord(kx_of(t, raw_k(t, g.n_freq, n, plo), ku), g);
      const double lhi = lattice_coord(kx_of(t, raw_k(t, g.n_freq, n, phi), ku), g);
      return (R)((lhi - llo) / 2.0);
    }
    default:
      return (R)1;
  }
}

// ES kernel exp(beta (sqrt(1 - z^2) - 1)) at a tap offset z in (-1, 1).  The taps the
// gridding uses satisfy |z| < 1 except on the measure-zero boundary z = -1 (fraction
// exactly W/2 - floor(W/2) from a cell), where this returns exp(-beta) ~ 1e-7 instead
// of 0.  FP32: hardware sqrt and exp2 (beta_l2e = beta log2 e).
__device__ __forceinline__ float es_kernel(float z, float beta_l2e) {
  const float s = fmaxf(fmaf(-z, z, 1.0f), 0.0f);
  return __builtin_amdgcn_exp2f(fmaf(beta_l2e, __builtin_amdgcn_sqrtf(s), -beta_l2e));
}
__device__ __forceinline__ double es_kernel(double z, double beta) {
  const double s = fmax(1.0 - z * z, 0.0);
  return exp(beta * (sqrt(s) - 1.0));
}
// the kernel-shape constant es_kernel expects for the compute type
template <typename R>
__device__ __forceinline__ R es_shape(const Geo& g) {
  return sizeof(R) == 4 ? (R)(g.beta * 1.4426950408889634) : (R)g.beta;
}

// Literal Algorithm-1 range gridding (Eq. (8)): a sample at lattice coordinate lam
// reaches the image-lattice points m with |m - lam| < q, with weight R_W(m - lam), the
// window's finite-interval transform.  On the M-point lattice row (M = image size) the
// sample sits at cell + fraction f = frac(tt) M, tt = kx fov_x / (2 pi M) cycles per
// pixel; the taps are d = k0 + i - f, k0 = floor(f - q) + 1, i < 2q (0 where |d| >= q:
// a sample on the lattice reaches 2q - 1 points).  One sincos(pi d0) serves every tap,
// since sin, cos(pi (d0 + i)) = (-1)^i sin, cos(pi d0).  FP64 taps; kept out of line.
__device__ __forceinline__ double lit_tap(double d, double sgn, double s0, double c0, double a, double ema2) {
  const double b = 2.0 * TFFR_PI * d;
  const double den = a * a + b * b;
  if (den == 0.0) return 1.0;
  return 2.0 * (a + ema2 * (b * (sgn * s0) - a * (sgn * c0))) / den;
}
template <typename R>
__device__ __attribute__((noinline)) void lit_spread(cplx<R>* buf, int N, double tt, double q, int ntaps, double a,
                                                     double ema2, cplx<R> c) {
  const double u = (tt - floor(tt)) * (double)N;
  const double fu = floor(u), fl = u - fu;
  const int k0 = (int)floor(fl - q) + 1;
  const int cell = (int)fu + k0;
  const double d0 = (double)k0 - fl;
  double s0, c0;
  sincospi(d0, &s0, &c0);
  for (int i = 0; i < ntaps; ++i) {
    const double d = d0 + (double)i;
    const R phi = fabs(d) < q ? (R)lit_tap(d, (i & 1) ? -1.0 : 1.0, s0, c0, a, ema2) : (R)0;
    cplx<R>& bb = buf[(cell + i) & (N - 1)];
    bb = bb + phi * c;
  }
}
template <typename R>
__device__ __attribute__((noinline)) cplx<R> lit_gather(const cplx<R>* buf, int N, double tt, double q, int ntaps,
                                                        double a, double ema2) {
  const double u = (tt - floor(tt)) * (double)N;
  const double fu = floor(u), fl = u - fu;
  const int k0 = (int)floor(fl - q) + 1;
  const int cell = (int)fu + k0;
  const double d0 = (double)k0 - fl;
  double s0, c0;
  sincospi(d0, &s0, &c0);
  cplx<R> acc = {0, 0};
  for (int i = 0; i < ntaps; ++i) {
    const double d = d0 + (double)i;
    const R phi = fabs(d) < q ? (R)lit_tap(d, (i & 1) ? -1.0 : 1.0, s0, c0, a, ema2) : (R)0;
    acc = acc + phi * buf[(cell + i) & (N - 1)];
  }
  return acc;
}

// Fine-grid position of a sample with lattice-per-pixel coordinate t (cycles per pixel):
// u = frac(t) n in [0, n), split in FP64 into an integer cell and a fraction.
template <typename R>
__device__ __forceinline__ void fine_pos(double t, int n, int& ui, R& f) {
  const double u = (t - floor(t)) * (double)n;
  const double fu = floor(u);
  ui = (int)fu;
  f = (R)(u - fu);
}

template <typename R>
__device__ __forceinline__ cplx<R> load_sample(const void* s, int stype, size_t i) {
  if (stype == ST_H2) {
    const half2s h = ((const half2s*)s)[i];
    return {(R)(float)h.x, (R)(float)h.y};
  }
  if (stype == ST_C128) {
    const cplx<double> v = ((const cplx<double>*)s)[i];
    return {(R)v.x, (R)v.y};
  }
  const cplx<float> v = ((const cplx<float>*)s)[i];
  return {(R)v.x, (R)v.y};
}

template <typename R>
__device__ __forceinline__ cplx<R> row_rotation(const Tab<R>& t, const R* phase, const R* dalong, int n) {
  R psi = 0;
  if (phase) psi += phase[n];
  if (dalong) psi += t.ky[n] * dalong[n];
  R sn, cs;
  if constexpr (sizeof(R) == 4) sincosf(psi, &sn, &cs);
  else sincos(psi, &sn, &cs);
  return {cs, sn};
}

// (D s)_p for plain FFR: the banded slice matrix applied around sample p (out of line).
template <typename R>
__device__ __attribute__((noinline)) cplx<R> ffr_apply(const void* samples, int stype, const R* w, size_t base, int p,
                                                       int n_freq, int r) {
  const R* drow = w + (base + p) * (2 * r + 1);
  cplx<R> acc = {0, 0};
  for (int o = -r; o <= r; ++o) {
    const int pp = p + o;
    if (pp >= 0 && pp < n_freq) acc = acc + drow[r + o] * load_sample<R>(samples, stype, base + pp);
  }
  return acc;
}

// Weighted, phased sample c[n,p] (forward input of the gridding); s is sample (n, p).
template <typename R>
__device__ __forceinline__ cplx<R> weighted_sample(const Geo& g, const Tab<R>& t, const float* poly, int stype,
                                                   const void* samples, const R* w, int n, int p,
                                                   double ku, double lam, cplx<R> rot, cplx<R> s) {
  const size_t base = (size_t)n * g.n_freq;
  if (g.weighting == 2)  // plain FFR: banded D within the slice
    return cmul(rot, ffr_apply<R>(samples, stype, w, base, p, g.n_freq, g.band_r));
  const R wt = w ? w[base + p] : diag_weight<R>(g, t, poly, ku, n, p, lam);
  return wt * cmul(rot, s);
}

// ============================================================================ forward
// Range stage: one azimuth slice per workgroup.  Spread the slice's weighted samples
// onto the periodic fine row, inverse FFT, keep the centred mx bins and divide by the
// kernel transform.  stage 0 dumps the gridded row instead.
//
// No atomics: kx grows along a slice, so when thread t takes the sample
// p = part start + block * S * NT + S t + j in sub-pass j, the samples of one sub-pass
// are S apart and their cell ranges are disjoint (the plan picks S with
// S * (smallest sample spacing) > W).  The slice is cut into parts whose span is less
// than the fine row, so no two samples of a part meet after wrapping.  Each sub-pass is
// a plain read-add-write into LDS followed by a barrier; the raw inputs of the next
// sub-pass are loaded while the current one is processed.
template <typename R, int LOGN, int NT, int SG>
__global__ __launch_bounds__(NT) void k_fwd_rows(Geo g, Tab<R> t, int stype, const void* __restrict__ samples,
                                                 const R* __restrict__ phase, const R* __restrict__ dalong,
                                                 const R* __restrict__ w, cplx<R>* __restrict__ out, int stage) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = (N + NT - 1) / NT;  // >= output bins per thread (mx <= N)
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  float* lpoly = reinterpret_cast<float*>(buf + N);
  const int n = blockIdx.x;
  const bool ffr = g.weighting == 2;
  const int S = g.sub, W = g.W, plen = g.part_len;
  const int nblk = (plen + S * NT - 1) / (S * NT);
  const size_t base = (size_t)n * g.n_freq;
  load_twiddles<N, NT>(tw, t.twx);
  const float* poly = load_poly<NT>(g, t.poly, lpoly);
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = {0, 0};
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  const R halfw = (R)(0.5 * g.W), inv_halfw = (R)(2.0 / g.W), beta = es_shape<R>(g);
  bool first = true;
  for (int pa = 0; pa < g.n_freq; pa += plen) {
    const int pb = min(pa + plen, g.n_freq);
    for (int blk = 0; blk < nblk; ++blk) {
      const int p0 = pa + blk * S * NT + S * (int)threadIdx.x;  // this thread's S consecutive samples
      for (int j0 = 0; j0 < S; j0 += SG) {
        // raw inputs of up to SG consecutive samples, loaded back to back
        double kr[SG];
        cplx<R> sr[SG];
#pragma unroll
        for (int j = 0; j < SG; ++j) {
          const int p = p0 + j0 + j;
          const bool ok = j0 + j < S && p < pb;
          kr[j] = ok ? raw_k(t, g.n_freq, n, p) : 0.0;
          sr[j] = (ok && !ffr) ? load_sample<R>(samples, stype, base + p) : cplx<R>{0, 0};
        }
        if (first) {
          __syncthreads();  // row zeroed, tables in LDS
          first = false;
        }
#pragma unroll
        for (int j = 0; j < SG; ++j) {
          if (j0 + j < S) {
            const int p = p0 + j0 + j;
            if (p < pb) {
              const double kx = kx_of(t, kr[j], ku);
              const double lam = lattice_coord(kx, g);
              const cplx<R> c = weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lam, rot, sr[j]);
              if (g.literal) {
                lit_spread<R>(buf, N, kx * g.tx_scale, g.q, g.lit_taps, g.a, g.ema2, c);
              } else {
                int ui;
                R f;
                fine_pos<R>(kx * g.tx_scale, N, ui, f);
                const int k0 = (int)ceil(f - halfw);
                const int cell = ui + k0;
                const R z0 = ((R)k0 - f) * inv_halfw;
                for (int i = 0; i < W; ++i) {
                  const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
                  cplx<R>& bb = buf[(cell + i) & (N - 1)];
                  bb = bb + phi * c;
                }
              }
            }
            __syncthreads();
          }
        }
      }
    }
  }
  if (first) __syncthreads();
  if (stage == 0) {
    for (int i = threadIdx.x; i < N; i += NT) out[(size_t)n * N + i] = buf[i];
    return;
  }
  const int mx = g.mx;
  R dx[DPT];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    dx[j] = jx < mx ? t.deapx[jx] : (R)0;
  }
  lds_fft<+1, N, NT, 1, 8, 1>(buf, tw);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    if (jx < mx) out[(size_t)n * mx + jx] = dx[j] * buf[(jx - mx / 2) & (N - 1)];
  }
}

// Range stage for densely sampled slices (the plan's choice when consecutive samples sit
// well under W fine cells apart).  Thread t takes the run of S consecutive samples
// p0 = part start + S t ... and slides a window of W register accumulators along the
// fine row: a sample whose first tap cell is c0 first retires the window cells below c0
// (in increasing cell order), then adds its W taps to the window at fixed register
// positions.  With S * (smallest sample spacing) > W, the first W cells a run retires
// (its "lead") are the only cells another run (the previous one) also reaches, so
// every other retired cell is read-add-written into LDS at once without conflict; the
// lead cells are kept in registers and added after one barrier, when no other run
// writes.  Two barriers per part instead of one per sample of a run.
template <typename R, int LOGN, int NT, int WM>
__global__ __launch_bounds__(NT) void k_fwd_rows_run(Geo g, Tab<R> t, int stype, const void* __restrict__ samples,
                                                     const R* __restrict__ phase, const R* __restrict__ dalong,
                                                     const R* __restrict__ w, cplx<R>* __restrict__ out,
                                                     int stage) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = (N + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  float* lpoly = reinterpret_cast<float*>(buf + N);
  const int n = blockIdx.x;
  const bool ffr = g.weighting == 2;
  const int S = g.sub, W = g.W, plen = g.part_len;
  const size_t base_s = (size_t)n * g.n_freq;
  load_twiddles<N, NT>(tw, t.twx);
  const float* poly = load_poly<NT>(g, t.poly, lpoly);
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = {0, 0};
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  const R halfw = (R)(0.5 * g.W), inv_halfw = (R)(2.0 / g.W), beta = es_shape<R>(g);
  __syncthreads();  // row zeroed, tables in LDS
  for (int pa = 0; pa < g.n_freq; pa += plen) {
    const int pb = min(pa + plen, g.n_freq);
    const int p0 = pa + S * (int)threadIdx.x;
    const int p1 = min(p0 + S, pb);
    cplx<R> acc[WM], lead[WM];
#pragma unroll
    for (int i = 0; i < WM; ++i) acc[i] = lead[i] = cplx<R>{0, 0};
    int base = 0, cfirst = 0;
    // retire the lowest window cell: into the lead registers if it is one of the run's
    // first W cells, else straight into the row; then shift the window down one cell
    auto retire = [&]() {
      if (base - cfirst < W) {
#pragma unroll
        for (int i = 0; i + 1 < WM; ++i) lead[i] = lead[i + 1];
        lead[WM - 1] = acc[0];
      } else {
        cplx<R>& bb = buf[base & (N - 1)];
        bb = bb + acc[0];
      }
#pragma unroll
      for (int i = 0; i + 1 < WM; ++i) acc[i] = acc[i + 1];
      acc[WM - 1] = cplx<R>{0, 0};
      ++base;
    };
    double k_nx = p0 < p1 ? raw_k(t, g.n_freq, n, p0) : 0.0;
    cplx<R> s_nx = (p0 < p1 && !ffr) ? load_sample<R>(samples, stype, base_s + p0) : cplx<R>{0, 0};
    for (int p = p0; p < p1; ++p) {
      const double kp = k_nx;
      const cplx<R> sp = s_nx;
      if (p + 1 < p1) {
        k_nx = raw_k(t, g.n_freq, n, p + 1);
        if (!ffr) s_nx = load_sample<R>(samples, stype, base_s + p + 1);
      }
      const double kx = kx_of(t, kp, ku);
      const double lam = lattice_coord(kx, g);
      const cplx<R> c = weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lam, rot, sp);
      const double tt = kx * g.tx_scale;
      int ui;
      R f;
      fine_pos<R>(tt, N, ui, f);
      const int k0 = (int)ceil(f - halfw);
      // unwrapped first tap cell (only differences and the low LOGN bits are used)
      const int c0 = (int)((unsigned)(int)floor(tt) * (unsigned)N + (unsigned)(ui + k0));
      if (p == p0) base = cfirst = c0;
      for (int adv = c0 - base; adv > 0; --adv) retire();
      const R z0 = ((R)k0 - f) * inv_halfw;
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        if (i < W) {
          const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
          acc[i] = acc[i] + phi * c;
        }
      }
    }
    if (p0 < p1)
      for (int i = 0; i < W; ++i) retire();
    __syncthreads();
    if (p0 < p1) {
#pragma unroll
      for (int i = 0; i < WM; ++i) {
        if (i >= WM - W) {
          cplx<R>& bb = buf[(cfirst + i - (WM - W)) & (N - 1)];
          bb = bb + lead[i];
        }
      }
    }
    __syncthreads();
  }
  if (stage == 0) {
    for (int i = threadIdx.x; i < N; i += NT) out[(size_t)n * N + i] = buf[i];
    return;
  }
  const int mx = g.mx;
  R dx[DPT];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    dx[j] = jx < mx ? t.deapx[jx] : (R)0;
  }
  lds_fft<+1, N, NT, 1, 16, 1>(buf, tw);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    if (jx < mx) out[(size_t)n * mx + jx] = dx[j] * buf[(jx - mx / 2) & (N - 1)];
  }
}

// ---------------------------------------------------------------------------- azimuth helpers
// The plan's azimuth cell table, entry e of fine cell iy at e * N + iy: the e-th (slice,
// tap) pair reaching the cell (padded with slice 0, tap 0).  A thread owns the cells
// threadIdx.x + j NT; its entries of one e are loaded together (coalesced over lanes).
template <typename R, int N, int NT>
struct CellEntries {
  int32_t n[N / NT];
  R w[N / NT];
};
template <typename R, int N, int NT>
__device__ __forceinline__ void load_entries(const Tab<R>& t, int e, CellEntries<R, N, NT>& ce) {
#pragma unroll
  for (int j = 0; j < N / NT; ++j) {
    const size_t i = (size_t)e * N + threadIdx.x + j * NT;
    ce.n[j] = t.ycell_n[i];
    ce.w[j] = t.ycell_w[i];
  }
}

// CB consecutive complex values, moved as one wide access where aligned
template <typename R, int CB>
struct alignas(CB * sizeof(cplx<R>) >= 16 ? 16 : CB * sizeof(cplx<R>)) CVec {
  cplx<R> v[CB];
};

// Stage the block's CB columns of the range spectra in LDS as hs[n][c] (zeros past the
// last column of the image).  A slice's CB values are one wide load when the block is
// full and the rows keep CB-alignment.  With one column per block (the largest images,
// several slices per thread) each slice is a separate row of the spectra, so a thread
// issues four slices' loads before storing any: one latency per batch, not per slice.
template <typename R, int NT, int CB>
__device__ __forceinline__ void stage_spectra(const Geo& g, const cplx<R>* __restrict__ hx, cplx<R>* hs, int c0,
                                              int ncol) {
  if constexpr (CB == 1) {
    constexpr int SU = 4;
    for (int n0 = threadIdx.x; n0 < g.n_pulses; n0 += SU * NT) {
      cplx<R> v[SU];
#pragma unroll
      for (int u = 0; u < SU; ++u) {
        const int nn = n0 + u * NT;
        v[u] = nn < g.n_pulses ? hx[(size_t)nn * g.mx + c0] : cplx<R>{0, 0};
      }
#pragma unroll
      for (int u = 0; u < SU; ++u)
        if (n0 + u * NT < g.n_pulses) hs[n0 + u * NT] = v[u];
    }
    return;
  }
  if (CB > 1 && ncol == CB && g.mx % CB == 0) {
    for (int nn = threadIdx.x; nn < g.n_pulses; nn += NT)
      *reinterpret_cast<CVec<R, CB>*>(hs + nn * CB) =
          *reinterpret_cast<const CVec<R, CB>*>(hx + (size_t)nn * g.mx + c0);
    return;
  }
  const int total = g.n_pulses * CB;
  for (int idx = threadIdx.x; idx < total; idx += NT) {
    const int nn = idx / CB, c = idx - nn * CB;
    hs[idx] = c < ncol ? hx[(size_t)nn * g.mx + c0 + c] : cplx<R>{0, 0};
  }
}

// Azimuth gridding of CB columns: every fine cell gathers its (slice, tap) pairs from the
// staged spectra (no atomics); buf[c][iy].  `cur` holds the thread's entries e = 0, and
// the entries e + 1 are loaded while those of e are applied.
template <typename R, int N, int NT, int CB>
__device__ __forceinline__ void cols_gather(const Geo& g, const Tab<R>& t, CellEntries<R, N, NT> cur,
                                            const cplx<R>* hs, cplx<R>* buf) {
  constexpr int CPT = N / NT;
  cplx<R> acc[CPT][CB];
#pragma unroll
  for (int j = 0; j < CPT; ++j)
#pragma unroll
    for (int c = 0; c < CB; ++c) acc[j][c] = {0, 0};
  const int E = g.yemax;
  for (int e = 0; e < E; ++e) {
    CellEntries<R, N, NT> nx = cur;
    if (e + 1 < E) load_entries(t, e + 1, nx);
#pragma unroll
    for (int j = 0; j < CPT; ++j)
#pragma unroll
      for (int c = 0; c < CB; ++c) acc[j][c] = acc[j][c] + cur.w[j] * hs[cur.n[j] * CB + c];
    cur = nx;
  }
#pragma unroll
  for (int j = 0; j < CPT; ++j)
#pragma unroll
    for (int c = 0; c < CB; ++c) buf[c * N + threadIdx.x + j * NT] = acc[j][c];
}

// Azimuth interpolation (type 2) of NC fine columns buf[c][.] at every slice: the W taps
// of slice n are loaded once and applied to all NC columns; column c goes to output
// array c / CS at image column c0 + c % CS (each array's CS columns as one wide store
// when the block is full and rows keep CS-alignment).
// A thread's first slice (n = threadIdx.x): its start cell and up to kRunWindow taps,
// loaded ahead (before the FFT that precedes the interpolation).
template <typename R>
struct SliceTaps {
  int ys;
  R tap[kRunWindow];
};
template <typename R>
__device__ __forceinline__ SliceTaps<R> load_slice(const Geo& g, const Tab<R>& t, int nn) {
  SliceTaps<R> f;
  f.ys = t.ystart[nn];
#pragma unroll
  for (int i = 0; i < kRunWindow; ++i) f.tap[i] = i < g.W ? t.ytap[(size_t)nn * g.W + i] : (R)0;
  return f;
}
template <typename R>
__device__ __forceinline__ SliceTaps<R> load_first_slice(const Geo& g, const Tab<R>& t) {
  return load_slice(g, t, min((int)threadIdx.x, g.n_pulses - 1));
}

// IL (interleaved, NC = 2 CS): a single output array [n_pulses][mx][2] takes column
// CS + c (first value) and column c (second value) of image column c0 + c, so each slice's
// block is one contiguous store of 2 CS values.
template <typename R, int N, int NT, int NC, int CS, bool IL = false>
__device__ __forceinline__ void cols_interp(const Geo& g, const Tab<R>& t, const cplx<R>* buf, int nc_valid,
                                            cplx<R>* const* out, int c0, const SliceTaps<R>& first) {
  const int W = g.W;
  const bool wide = CS > 1 && nc_valid == CS && g.mx % CS == 0;
  for (int nn = threadIdx.x; nn < g.n_pulses; nn += NT) {
    cplx<R> acc[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[c] = {0, 0};
    if (nn == (int)threadIdx.x && W <= kRunWindow) {  // the prefetched first slice
#pragma unroll
      for (int i = 0; i < kRunWindow; ++i) {
        if (i < W) {
          const int cell = (first.ys + i) & (N - 1);
#pragma unroll
          for (int c = 0; c < NC; ++c) acc[c] = acc[c] + first.tap[i] * buf[c * N + cell];
        }
      }
    } else {
      const int ys = t.ystart[nn];
      const R* tap = t.ytap + (size_t)nn * W;
      for (int i = 0; i < W; ++i) {
        const R tp = tap[i];
        const int cell = (ys + i) & (N - 1);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = acc[c] + tp * buf[c * N + cell];
      }
    }
    if constexpr (IL) {
      cplx<R>* o = out[0] + ((size_t)nn * g.mx + c0) * 2;
      if (nc_valid == CS) {
        CVec<R, 2 * CS> v;
#pragma unroll
        for (int c = 0; c < CS; ++c) {
          v.v[2 * c] = acc[CS + c];
          v.v[2 * c + 1] = acc[c];
        }
        *reinterpret_cast<CVec<R, 2 * CS>*>(o) = v;
      } else {
#pragma unroll
        for (int c = 0; c < CS; ++c)
          if (c < nc_valid) {
            o[2 * c] = acc[CS + c];
            o[2 * c + 1] = acc[c];
          }
      }
    } else if (wide) {
#pragma unroll
      for (int o = 0; o < NC / CS; ++o) {
        CVec<R, CS> v;
#pragma unroll
        for (int c = 0; c < CS; ++c) v.v[c] = acc[o * CS + c];
        *reinterpret_cast<CVec<R, CS>*>(out[o] + (size_t)nn * g.mx + c0) = v;
      }
    } else {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if ((c % CS) < nc_valid) out[c / CS][(size_t)nn * g.mx + c0 + (c % CS)] = acc[c];
    }
  }
}

// Azimuth stage: CB range columns per workgroup.  The block's columns of the range
// spectra are staged in LDS; every fine azimuth cell gathers its (slice, tap) pairs for
// all CB columns at once (no atomics), batched inverse FFT along azimuth, keep the
// centred my bins, divide by the kernel transform, write the image columns
// (range-major).  With partials non-null the block also writes its share of the
// image-entropy sums (sum |I|^2, sum |I|^2 ln |I|^2).
template <typename R, int LOGN, int NT, int CB>
__global__ __launch_bounds__(NT) void k_fwd_cols(Geo g, Tab<R> t, const cplx<R>* __restrict__ hx,
                                                 cplx<R>* __restrict__ img, double* __restrict__ partials) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = N / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  cplx<R>* hs = buf + (size_t)CB * N;  // [n_pulses][CB]
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int c0 = lb * CB;
  const int ncol = min(CB, g.mx - c0);
  const int my = g.my;
  CellEntries<R, N, NT> ce;
  load_entries(t, 0, ce);
  load_twiddles<N, NT>(tw, t.twy);
  stage_spectra<R, NT, CB>(g, hx, hs, c0, ncol);
  R dy[DPT];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jy = threadIdx.x + j * NT;
    dy[j] = jy < my ? t.deapy[jy] : (R)0;
  }
  __syncthreads();
  cols_gather<R, N, NT, CB>(g, t, ce, hs, buf);
  __syncthreads();
  lds_fft<+1, N, NT, CB, 8, 1>(buf, tw);
  double es = 0.0, et = 0.0;
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    if (c < ncol) {
      const cplx<R>* col = buf + c * N;
      cplx<R>* o = img + (size_t)(c0 + c) * my;
#pragma unroll
      for (int j = 0; j < DPT; ++j) {
        const int jy = threadIdx.x + j * NT;
        if (jy < my) {
          const cplx<R> v = dy[j] * col[(jy - my / 2) & (N - 1)];
          o[jy] = v;
          if (partials) {
            const R a = v.x * v.x + v.y * v.y;
            es += (double)a;
            if (a > (R)0) et += (double)(a * log(a));
          }
        }
      }
    }
  }
  if (partials) {
    es = block_sum<NT>(es);
    et = block_sum<NT>(et);
    if (threadIdx.x == 0) {
      partials[2 * lb] = es;
      partials[2 * lb + 1] = et;
    }
  }
}

// Entropy step, azimuth stage forward and backward in one pass per column block.  The
// entropy gradient is linear in two local fields,
//   dE/dI = -(2/S)(ln|I|^2 - ln S + E) I = alpha I (ln|I|^2 - cc) + (beta + alpha cc) I,
// alpha = -2/S, beta = 2 T / S^2 (S = sum |I|^2, T = sum |I|^2 ln |I|^2 over the whole
// image, E = ln S - T/S), for any constant cc.  So the block, right after forming its
// image columns (written out, with its entropy partial sums), takes the adjoint azimuth
// transform of both fields, I (ln|I|^2 - cc) -> h1 and I -> h2, with cc = ln of the
// block's mean |I|^2 (keeps the first field centred; stored in cblk), and the range
// adjoint combines alpha h1 + (beta + alpha cc) h2 once the global sums are known.
// LDS: the two fields' fine columns [2][CB][N] reuse the staged-spectra space.  h12 is
// [n_pulses][mx][2]: h1 and h2 of each image column interleaved, so a slice's values of
// the block are one contiguous store.
template <typename R, int LOGN, int NT, int CB>
__global__ __launch_bounds__(NT) void k_ent_cols(Geo g, Tab<R> t, const cplx<R>* __restrict__ hx,
                                                 cplx<R>* __restrict__ img, double* __restrict__ partials,
                                                 R* __restrict__ cblk, cplx<R>* __restrict__ h12) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = N / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();  // [CB][N]: image field I, then its transform
  cplx<R>* hs = buf + (size_t)CB * N;   // staged spectra; afterwards [CB][N] the field I (ln|I|^2 - cc)
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int c0 = lb * CB;
  const int ncol = min(CB, g.mx - c0);
  const int my = g.my;
  // everything this block loads from tables is requested up front: cell entries,
  // deapodisation factors of its pixels, the first slice's interpolation taps
  CellEntries<R, N, NT> ce;
  load_entries(t, 0, ce);
  R dyv[DPT];
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int i = threadIdx.x + j * NT;
    const int jy = (i < N / 2 ? i : i - N) + my / 2;
    dyv[j] = (jy >= 0 && jy < my) ? t.deapy[jy] : (R)0;
  }
  const SliceTaps<R> first = load_first_slice(g, t);
  load_twiddles<N, NT>(tw, t.twy);
  stage_spectra<R, NT, CB>(g, hx, hs, c0, ncol);
  __syncthreads();
  cols_gather<R, N, NT, CB>(g, t, ce, hs, buf);
  __syncthreads();
  lds_fft<+1, N, NT, CB, 8, 1>(buf, tw);
  // image pixels: thread owns fine bins i = threadIdx.x + j NT (pixel jy = signed(i) + my/2)
  double es = 0.0, et = 0.0;
  cplx<R> v[CB][DPT];
  R lg[CB][DPT];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int i = threadIdx.x + j * NT;
      const int jy = (i < N / 2 ? i : i - N) + my / 2;
      v[c][j] = {0, 0};
      lg[c][j] = 0;
      if (c < ncol && jy >= 0 && jy < my) {
        const cplx<R> x = dyv[j] * buf[c * N + i];
        img[(size_t)(c0 + c) * my + jy] = x;
        const R a = x.x * x.x + x.y * x.y;
        es += (double)a;
        if (a > (R)0) {
          lg[c][j] = log(a);
          et += (double)(a * lg[c][j]);
          v[c][j] = x;
        }
      }
    }
  }
  es = block_sum<NT>(es);  // (its barriers also end every read of buf and hs above)
  et = block_sum<NT>(et);
  const double npix = (double)ncol * (double)my;
  const R cc = es > 0.0 ? (R)log(es / npix) : (R)0;
  if (threadIdx.x == 0) {
    partials[2 * lb] = es;
    partials[2 * lb + 1] = et;
    cblk[lb] = cc;
  }
  // adjoint fields, deapodised and zero-padded on the fine grid (same bins as above)
#pragma unroll
  for (int c = 0; c < CB; ++c) {
#pragma unroll
    for (int j = 0; j < DPT; ++j) {
      const int i = threadIdx.x + j * NT;
      const cplx<R> x = dyv[j] * v[c][j];
      buf[c * N + i] = x;
      hs[c * N + i] = (lg[c][j] - cc) * x;
    }
  }
  __syncthreads();
  lds_fft<-1, N, NT, 2 * CB, 8, 2>(buf, tw);  // buf and hs are contiguous: 2 CB columns
  cplx<R>* outs[1] = {h12};
  cols_interp<R, N, NT, 2 * CB, CB, true>(g, t, buf, ncol, outs, c0, first);
}

// Image entropy from the per-block sums: E = ln S - (1/S) sum a ln a.  One block.
// stats[0] = S, stats[1] = E; *loss = E.
template <int NT>
__global__ __launch_bounds__(NT) void k_entropy_stats(const double* __restrict__ partials, int nparts,
                                                      double* __restrict__ stats, double* __restrict__ loss) {
  double s = 0.0, tl = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) {
    s += partials[2 * i];
    tl += partials[2 * i + 1];
  }
  s = block_sum<NT>(s);
  tl = block_sum<NT>(tl);
  if (threadIdx.x == 0) {
    const double E = (s > 0.0) ? log(s) - tl / s : 0.0;
    stats[0] = s;
    stats[1] = E;
    if (loss) *loss = E;
  }
}

// ============================================================================ adjoint
// Azimuth stage, type 2: per range column, divide by the kernel transform, zero-pad to
// the fine grid, forward FFT (sign -, batched over the CB columns), and interpolate at
// every slice's azimuth position.  Entropy mode: `cot` is the image I itself and the
// cotangent is the entropy gradient -(2/S)(ln |I|^2 - ln S + E) I (0 where I = 0),
// formed in registers, with (S, E) read from stats, or reduced by the block itself from
// the forward kernel's nparts partial sums (then block 0 also writes *loss).
template <typename R, int LOGN, int NT, int CB>
__global__ __launch_bounds__(NT) void k_adj_cols(Geo g, Tab<R> t, const cplx<R>* __restrict__ cot,
                                                 cplx<R>* __restrict__ hx, const double* __restrict__ stats,
                                                 const double* __restrict__ partials, int nparts,
                                                 double* __restrict__ loss) {
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
  const int ncol = min(CB, g.mx - c0);
  const int my = g.my;
  load_twiddles<N, NT>(tw, t.twy);
  R sc = 0, off = 0;
  const bool ent = stats || partials;
  if (partials) {
    double es = 0.0, et = 0.0;
    for (int i = threadIdx.x; i < nparts; i += NT) {
      es += partials[2 * i];
      et += partials[2 * i + 1];
    }
    es = block_sum<NT>(es);
    et = block_sum<NT>(et);
    const double E = (es > 0.0) ? log(es) - et / es : 0.0;
    if (loss && blockIdx.x == 0 && threadIdx.x == 0) *loss = E;
    sc = (R)(-2.0 / es);
    off = (R)(E - log(es));
  } else if (stats) {
    sc = (R)(-2.0 / stats[0]);
    off = (R)(stats[1] - log(stats[0]));
  }
  for (int idx = threadIdx.x; idx < CB * N; idx += NT) {
    const int c = idx / N, i = idx - c * N;
    const int jp = i < N / 2 ? i : i - N;  // signed bin
    const int jy = jp + my / 2;
    cplx<R> v = {0, 0};
    if (c < ncol && jy >= 0 && jy < my) {
      v = cot[(size_t)(c0 + c) * my + jy];
      if (ent) {
        const R a = v.x * v.x + v.y * v.y;
        v = a > (R)0 ? (sc * (log(a) + off)) * v : cplx<R>{0, 0};
      }
      v = t.deapy[jy] * v;
    }
    buf[idx] = v;
  }
  __syncthreads();
  const SliceTaps<R> first = load_first_slice(g, t);
  lds_fft<-1, N, NT, CB, 8, 1>(buf, tw);
  cplx<R>* outs[1] = {hx};
  cols_interp<R, N, NT, CB, CB>(g, t, buf, ncol, outs, c0, first);
}

// Range stage, type 2: per slice, divide by the kernel transform, zero-pad, forward FFT
// (sign -), interpolate at every sample, apply D^T and exp(-i psi), and reduce the
// per-slice phase gradient sum_p Re(conj(g'_p) i s'_p) = sum_p (g_i s_r - g_r s_i).
// The raw inputs of a thread's first sample are loaded before the FFT, and those of
// the next sample while the current one is processed.
template <typename R, int LOGN, int NT>
__global__ __launch_bounds__(NT) void k_adj_rows(Geo g, Tab<R> t, int stype, const cplx<R>* __restrict__ hx,
                                                 const void* __restrict__ samples, const R* __restrict__ phase,
                                                 const R* __restrict__ dalong, const R* __restrict__ w,
                                                 cplx<R>* __restrict__ grad_s, R* __restrict__ grad_phase,
                                                 R* __restrict__ grad_dalong, EntComb<R> ec) {
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  float* lpoly = reinterpret_cast<float*>(buf + N);
  cplx<R>* gbuf = reinterpret_cast<cplx<R>*>(lpoly + kPolyLds);  // FFR only: interpolated values
  const int n = blockIdx.x;
  const int mx = g.mx;
  const size_t base = (size_t)n * g.n_freq;
  const bool ffr = g.weighting == 2;
  const bool want_phase = grad_phase || grad_dalong;
  const bool need_s = want_phase && !ffr;
  int p_next = threadIdx.x;
  double k_next = p_next < g.n_freq ? raw_k(t, g.n_freq, n, p_next) : 0.0;
  cplx<R> s_next = (need_s && p_next < g.n_freq) ? load_sample<R>(samples, stype, base + p_next) : cplx<R>{0, 0};
  R w_next = (w && !ffr && p_next < g.n_freq) ? w[base + p_next] : (R)0;
  load_twiddles<N, NT>(tw, t.twx);
  const float* poly = load_poly<NT>(g, t.poly, lpoly);
  const cplx<R>* in = hx + (size_t)n * mx;
  if (ec.h12) {
    // entropy step: the range-spectra cotangent is alpha h1 + (beta + alpha cc[col block]) h2
    double S, T;
    if (ec.partials) {
      double es = 0.0, et = 0.0;
      for (int i = threadIdx.x; i < ec.nparts; i += NT) {
        es += ec.partials[2 * i];
        et += ec.partials[2 * i + 1];
      }
      S = block_sum<NT>(es);
      T = block_sum<NT>(et);
      if (ec.loss && n == 0 && threadIdx.x == 0) *ec.loss = S > 0.0 ? log(S) - T / S : 0.0;
    } else {
      S = ec.stats[0];
      T = S > 0.0 ? S * (log(S) - ec.stats[1]) : 0.0;
    }
    const double al = S > 0.0 ? -2.0 / S : 0.0, be = S > 0.0 ? 2.0 * T / (S * S) : 0.0;
    const CVec<R, 2>* in12 = reinterpret_cast<const CVec<R, 2>*>(ec.h12) + (size_t)n * mx;
    for (int i = threadIdx.x; i < N; i += NT) {
      const int jp = i < N / 2 ? i : i - N;
      const int jx = jp + mx / 2;
      cplx<R> v = {0, 0};
      if (jx >= 0 && jx < mx) {
        const R c2 = (R)(be + al * (double)ec.cblk[jx / ec.cb]);
        const CVec<R, 2> f = in12[jx];
        v = t.deapx[jx] * ((R)al * f.v[0] + c2 * f.v[1]);
      }
      buf[i] = v;
    }
  } else {
    for (int i = threadIdx.x; i < N; i += NT) {
      const int jp = i < N / 2 ? i : i - N;
      const int jx = jp + mx / 2;
      buf[i] = (jx >= 0 && jx < mx) ? t.deapx[jx] * in[jx] : cplx<R>{0, 0};
    }
  }
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  const R halfw = (R)(0.5 * g.W), inv_halfw = (R)(2.0 / g.W), beta = es_shape<R>(g);
  __syncthreads();
  lds_fft<-1, N, NT, 1, 8, 1>(buf, tw);
  double acc_phase = 0.0;
  for (int p = threadIdx.x; p < g.n_freq; p += NT) {
    const double kp = k_next;
    const cplx<R> sp = s_next;
    const R wp = w_next;
    p_next = p + NT;
    if (p_next < g.n_freq) {
      k_next = raw_k(t, g.n_freq, n, p_next);
      if (need_s) s_next = load_sample<R>(samples, stype, base + p_next);
      if (w && !ffr) w_next = w[base + p_next];
    }
    const double kx = kx_of(t, kp, ku);
    cplx<R> a = {0, 0};
    if (g.literal) {
      a = lit_gather<R>(buf, N, kx * g.tx_scale, g.q, g.lit_taps, g.a, g.ema2);
    } else {
      int ui;
      R f;
      fine_pos<R>(kx * g.tx_scale, N, ui, f);
      const int k0 = (int)ceil(f - halfw);
      const int cell = ui + k0;
      const R z0 = ((R)k0 - f) * inv_halfw;
      for (int i = 0; i < g.W; ++i) {
        const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
        a = a + phi * buf[(cell + i) & (N - 1)];
      }
    }
    if (ffr) {
      gbuf[p] = a;
      continue;
    }
    const R wt = w ? wp : diag_weight<R>(g, t, poly, ku, n, p, lattice_coord(kx, g));
    const cplx<R> gs = cmulc(wt * a, rot);  // exp(-i psi) D^T A^H
    grad_s[base + p] = gs;
    if (want_phase) acc_phase += (double)gs.y * (double)sp.x - (double)gs.x * (double)sp.y;
  }
  if (ffr) {
    __syncthreads();
    const int r = g.band_r;
    for (int p = threadIdx.x; p < g.n_freq; p += NT) {
      cplx<R> a = {0, 0};
      for (int o = -r; o <= r; ++o) {  // (D^T x)_p = sum_o D_{p+o, p} x_{p+o}
        const int pp = p + o;
        if (pp >= 0 && pp < g.n_freq) a = a + w[(base + pp) * (2 * r + 1) + (r - o)] * gbuf[pp];
      }
      const cplx<R> gs = cmulc(a, rot);
      grad_s[base + p] = gs;
      if (want_phase) {
        const cplx<R> sv = load_sample<R>(samples, stype, base + p);
        acc_phase += (double)gs.y * (double)sv.x - (double)gs.x * (double)sv.y;
      }
    }
  }
  if (want_phase) {
    const double tot = block_sum<NT>(acc_phase);
    if (threadIdx.x == 0) {
      if (grad_phase) grad_phase[n] = (R)tot;
      if (grad_dalong) grad_dalong[n] = (R)((double)t.ky[n] * tot);
    }
  }
}

// Per-slice phase and position gradients from a sample cotangent g (w.r.t. the raw
// samples s): dL/dphi_n = sum_p Re(conj(g) i s) = sum_p (Im g Re s - Re g Im s), FP64
// accumulation, one workgroup per slice; dL/d(du_n) = ky_n dL/dphi_n.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_row_phase_grad(Geo g, Tab<R> t, int stype, const void* __restrict__ samples,
                                                       const cplx<R>* __restrict__ grad_s, R* __restrict__ grad_phase,
                                                       R* __restrict__ grad_dalong) {
  const int n = blockIdx.x;
  const size_t base = (size_t)n * g.n_freq;
  double acc = 0.0;
  for (int p = threadIdx.x; p < g.n_freq; p += NT) {
    const cplx<R> sv = load_sample<R>(samples, stype, base + p);
    const cplx<R> gv = grad_s[base + p];
    acc += (double)gv.y * (double)sv.x - (double)gv.x * (double)sv.y;
  }
  const double tot = block_sum<NT>(acc);
  if (threadIdx.x == 0) {
    grad_phase[n] = (R)tot;
    if (grad_dalong) grad_dalong[n] = (R)((double)t.ky[n] * tot);
  }
}

// ============================================================================ coordinate gradients
// dL/dkx[n,p] = Re(i c conj(A^H(X G))[n,p]) and dL/dky[n] = sum_p Re(i c conj(A^H(Y G))[n,p])
// for a cotangent G, the weights held fixed (c = weighted, phased sample; X, Y pixel
// coordinates).  The X weight is constant along an image column, so it is applied in the
// range stage; the azimuth stage transforms the two fields G and Y G together.
//
// Azimuth stage: per column block, fields f0 = G, f1 = Y G (deapodised, zero-padded),
// batched forward FFT over the 2 CB columns, interpolation at every slice -> h0, h1.
template <typename R, int LOGN, int NT, int CB>
__global__ __launch_bounds__(NT) void k_coord_cols(Geo g, Tab<R> t, const cplx<R>* __restrict__ cot,
                                                   cplx<R>* __restrict__ h0, cplx<R>* __restrict__ h1) {
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();  // [2][CB][N]
  const int c0 = xcd_block(blockIdx.x, gridDim.x) * CB;
  const int ncol = min(CB, g.mx - c0);
  const int my = g.my;
  const R ypix = (R)g.fov_y / (R)my;
  load_twiddles<N, NT>(tw, t.twy);
  for (int idx = threadIdx.x; idx < CB * N; idx += NT) {
    const int c = idx / N, i = idx - c * N;
    const int jp = i < N / 2 ? i : i - N;  // signed bin
    const int jy = jp + my / 2;
    cplx<R> v = {0, 0};
    if (c < ncol && jy >= 0 && jy < my) v = t.deapy[jy] * cot[(size_t)(c0 + c) * my + jy];
    buf[idx] = v;
    buf[CB * N + idx] = ((R)jp * ypix) * v;
  }
  __syncthreads();
  const SliceTaps<R> first = load_first_slice(g, t);
  lds_fft<-1, N, NT, 2 * CB>(buf, tw);
  cplx<R>* outs[2] = {h0, h1};
  cols_interp<R, N, NT, 2 * CB, CB>(g, t, buf, ncol, outs, c0, first);
}

// Range stage: per slice, rows X h0 and h1 (deapodised, zero-padded), batched forward
// FFT, and at every sample both interpolations with one set of taps; the weighted,
// phased sample c is formed as in the forward path.  FP64 reduction of dL/dky per slice.
template <typename R, int LOGN, int NT>
__global__ __launch_bounds__(NT) void k_coord_rows(Geo g, Tab<R> t, int stype, const cplx<R>* __restrict__ h0,
                                                   const cplx<R>* __restrict__ h1, const void* __restrict__ samples,
                                                   const R* __restrict__ phase, const R* __restrict__ dalong,
                                                   const R* __restrict__ w, R* __restrict__ grad_kx,
                                                   R* __restrict__ grad_ky) {
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();  // [2][N]
  float* lpoly = reinterpret_cast<float*>(buf + 2 * N);
  const int n = blockIdx.x;
  const int mx = g.mx;
  const size_t base = (size_t)n * g.n_freq;
  const bool ffr = g.weighting == 2;
  const R xpix = (R)g.fov_x / (R)mx;
  load_twiddles<N, NT>(tw, t.twx);
  const float* poly = load_poly<NT>(g, t.poly, lpoly);
  for (int i = threadIdx.x; i < N; i += NT) {
    const int jp = i < N / 2 ? i : i - N;
    const int jx = jp + mx / 2;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (jx >= 0 && jx < mx) {
      a = (t.deapx[jx] * ((R)jp * xpix)) * h0[(size_t)n * mx + jx];
      b = t.deapx[jx] * h1[(size_t)n * mx + jx];
    }
    buf[i] = a;
    buf[N + i] = b;
  }
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  const R halfw = (R)(0.5 * g.W), inv_halfw = (R)(2.0 / g.W), beta = es_shape<R>(g);
  __syncthreads();
  lds_fft<-1, N, NT, 2>(buf, tw);
  double acc_ky = 0.0;
  for (int p = threadIdx.x; p < g.n_freq; p += NT) {
    const double kx = kx_of(t, raw_k(t, g.n_freq, n, p), ku);
    const cplx<R> sp = ffr ? cplx<R>{0, 0} : load_sample<R>(samples, stype, base + p);
    const cplx<R> c = weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lattice_coord(kx, g), rot, sp);
    cplx<R> ax = {0, 0}, ay = {0, 0};
    if (g.literal) {
      ax = lit_gather<R>(buf, N, kx * g.tx_scale, g.q, g.lit_taps, g.a, g.ema2);
      ay = lit_gather<R>(buf + N, N, kx * g.tx_scale, g.q, g.lit_taps, g.a, g.ema2);
    } else {
      int ui;
      R f;
      fine_pos<R>(kx * g.tx_scale, N, ui, f);
      const int k0 = (int)ceil(f - halfw);
      const int cell = ui + k0;
      const R z0 = ((R)k0 - f) * inv_halfw;
      for (int i = 0; i < g.W; ++i) {
        const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
        const int ci = (cell + i) & (N - 1);
        ax = ax + phi * buf[ci];
        ay = ay + phi * buf[N + ci];
      }
    }
    // Re(i c conj(a)) = Re(c) Im(a) - Im(c) Re(a)
    grad_kx[base + p] = c.x * ax.y - c.y * ax.x;
    acc_ky += (double)c.x * (double)ay.y - (double)c.y * (double)ay.x;
  }
  const double tot = block_sum<NT>(acc_ky);
  if (threadIdx.x == 0) grad_ky[n] = (R)tot;
}

// ============================================================================ weights
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_weights(Geo g, Tab<R> t, R* __restrict__ w,
                                                unsigned long long* __restrict__ kept_partial) {
  const size_t total = (size_t)g.n_pulses * g.n_freq;
  unsigned long long kept = 0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < total; i += (size_t)gridDim.x * NT) {
    const int n = (int)(i / g.n_freq), p = (int)(i - (size_t)n * g.n_freq);
    const double ku = t.ku[n];
    const double lam = lattice_coord(kx_of(t, raw_k(t, g.n_freq, n, p), ku), g);
    const R v = diag_weight<R>(g, t, t.poly, ku, n, p, lam);
    if (w) w[i] = v;
    kept += (v != (R)0) ? 1ull : 0ull;
  }
  const double tot = block_sum<NT>((double)kept);
  if (threadIdx.x == 0 && kept_partial) kept_partial[blockIdx.x] = (unsigned long long)tot;
}

__global__ void k_sum_u64(const unsigned long long* __restrict__ parts, int n, long long* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int i = 0; i < n; ++i) s += parts[i];
    *out = (long long)s;
  }
}

// ============================================================================ plain FFR
// Per sample p and tap k in [-K, K] (K = ceil(q) + 1): R_Psi and R_W at d = k - delta_p,
// zero where |d| >= q.  Both transforms need sin and cos of pi d = pi k - pi delta, so
// one sincos(pi delta) per sample serves every tap: sin(pi d) = -(-1)^k sin(pi delta),
// cos(pi d) = (-1)^k cos(pi delta).
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_ffr_taps(Geo g, Tab<R> t, double* __restrict__ tpsi, double* __restrict__ tw,
                                                 int* __restrict__ fl) {
  const size_t total = (size_t)g.n_pulses * g.n_freq;
  const int K = (int)ceil(g.q) + 1, KT = 2 * K + 1;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < total; i += (size_t)gridDim.x * NT) {
    const int n = (int)(i / g.n_freq), p = (int)(i - (size_t)n * g.n_freq);
    const double lam = lattice_coord(kx_of(t, raw_k(t, g.n_freq, n, p), t.ku[n]), g);
    const double f = floor(lam), delta = lam - f;
    fl[i] = (int)f;
    double sd, cd;
    sincospi(delta, &sd, &cd);
    for (int k = -K; k <= K; ++k) {
      const double d = (double)k - delta;
      double vp = 0.0, vw = 0.0;
      if (fabs(d) < g.q) {
        const double sg = (k & 1) ? -1.0 : 1.0;
        const double sn = -sg * sd, cs = sg * cd;  // sin, cos of pi d = b / 2
        const double b = 2.0 * TFFR_PI * d, den = g.a * g.a + b * b;
        if (den == 0.0) {
          vp = vw = 1.0;
        } else {
          vw = 2.0 * (g.a + g.ema2 * (b * sn - g.a * cs)) / den;
          vp = 2.0 * (g.epa2 * (b * sn + g.a * cs) - g.a) / den;
        }
      }
      tpsi[i * KT + (k + K)] = vp;
      tw[i * KT + (k + K)] = vw;
    }
  }
}

// Band of the truncated frame product of every slice, row p, columns p-b..p+b:
// G~_{p,p'} = sum over integers m with |m - lam_p| < q and |m - lam_p'| < q of
// R_Psi(m - lam_p) R_W(m - lam_p'), from the per-sample tap tables.
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_ffr_build(Geo g, const double* __restrict__ tpsi,
                                                  const double* __restrict__ tw, const int* __restrict__ fl,
                                                  double* __restrict__ gband) {
  const int b = g.band_b, wdt = 2 * b + 1;
  const size_t total = (size_t)g.n_pulses * g.n_freq;
  const int K = (int)ceil(g.q) + 1, KT = 2 * K + 1;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < total; i += (size_t)gridDim.x * NT) {
    const int n = (int)(i / g.n_freq), p = (int)(i - (size_t)n * g.n_freq);
    const int fp = fl[i];
    for (int o = -b; o <= b; ++o) {
      const int pp = p + o;
      double acc = 0.0;
      if (pp >= 0 && pp < g.n_freq) {
        const size_t j = i + o;
        const int sh = fp - fl[j];  // m = fp + k = fl[pp] + (k + sh)
        for (int k = -K; k <= K; ++k) {
          const int k2 = k + sh;
          if (k2 >= -K && k2 <= K) acc += tpsi[i * KT + (k + K)] * tw[j * KT + (k2 + K)];
        }
      }
      gband[i * wdt + (b + o)] = acc;
    }
  }
}

// One workgroup per slice: the slice's band is loaded into LDS (coalesced), then one
// lane runs LU without pivoting of the banded frame product (half bandwidth B) in
// place, then the band of its inverse by the Takahashi recurrences (UZ = L^-1 for the
// upper part, ZL = U^-1 for the lower part, which close within the band), and writes
// B_r of the inverse (= pinv for a full-rank product).  Both sequential sweeps keep a
// sliding window of the band in registers and read the factors from LDS.  status[0] is
// set to 1 on a vanishing pivot (D is then zero).
template <typename R, int B>
__global__ __launch_bounds__(64) void k_ffr_solve(Geo g, const double* __restrict__ gband, R* __restrict__ dband,
                                                  int* __restrict__ status) {
  constexpr int WD = 2 * B + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  double* F = reinterpret_cast<double*>(smem);  // [P][WD]: A, then L (o < 0) and U (o >= 0) in place
  const int n = blockIdx.x;
  const int P = g.n_freq, r = g.band_r;
  const double* A = gband + (size_t)n * P * WD;
  for (int e = threadIdx.x; e < P * WD; e += 64) F[e] = A[e];
  __syncthreads();
  if (threadIdx.x != 0) return;
  R* D = dband + (size_t)n * P * (2 * r + 1);
  auto f_at = [&](int i, int j) -> double {
    return (i < P && j < P && j - i >= -B && j - i <= B) ? F[i * WD + B + (j - i)] : 0.0;
  };
  double scale = 0.0;
  for (int i = 0; i < P; ++i) scale = fmax(scale, fabs(F[i * WD + B]));
  // ---- LU: window M[rr][c] = A(k + rr, k + c)
  double M[B + 1][B + 1];
#pragma unroll
  for (int rr = 0; rr <= B; ++rr)
#pragma unroll
    for (int c = 0; c <= B; ++c) M[rr][c] = f_at(rr, c);
  bool bad = false;
  for (int k = 0; k < P; ++k) {
    // entries entering the window after this step (untouched by steps <= k)
    double nrow[B + 1], ncol[B];
#pragma unroll
    for (int c = 0; c <= B; ++c) nrow[c] = f_at(k + B + 1, k + 1 + c);
#pragma unroll
    for (int rr = 0; rr < B; ++rr) ncol[rr] = f_at(k + 1 + rr, k + B + 1);
    const double piv = M[0][0];
    if (!(fabs(piv) > 1e-12 * scale)) {
      bad = true;
      break;
    }
    const double inv = 1.0 / piv;
#pragma unroll
    for (int c = 0; c <= B; ++c)
      if (k + c < P) F[k * WD + B + c] = M[0][c];
    double l[B + 1];
#pragma unroll
    for (int rr = 1; rr <= B; ++rr) {
      l[rr] = M[rr][0] * inv;
      if (k + rr < P) F[(k + rr) * WD + B - rr] = l[rr];
    }
#pragma unroll
    for (int rr = 1; rr <= B; ++rr)
#pragma unroll
      for (int c = 1; c <= B; ++c) M[rr][c] -= l[rr] * M[0][c];
#pragma unroll
    for (int rr = 0; rr < B; ++rr)
#pragma unroll
      for (int c = 0; c < B; ++c) M[rr][c] = M[rr + 1][c + 1];
#pragma unroll
    for (int c = 0; c <= B; ++c) M[B][c] = nrow[c];
#pragma unroll
    for (int rr = 0; rr < B; ++rr) M[rr][B] = ncol[rr];
  }
  if (bad) {
    atomicExch(status, 1);
    for (int e = 0; e < P * (2 * r + 1); ++e) D[e] = (R)0;
    return;
  }
  // ---- selected inversion, i = P-1 .. 0: window ZW[rr][o] = Z(i+1+rr, i+1+rr+o-B)
  double ZW[B][WD];
#pragma unroll
  for (int rr = 0; rr < B; ++rr)
#pragma unroll
    for (int o = 0; o < WD; ++o) ZW[rr][o] = 0.0;
  for (int i = P - 1; i >= 0; --i) {
    double U[B + 1];
#pragma unroll
    for (int c = 0; c <= B; ++c) U[c] = (i + c < P) ? F[i * WD + B + c] : 0.0;
    double Lv[B + 1][B];  // Lv[c][dk] = L(j + 1 + dk, j), j = i - c
#pragma unroll
    for (int c = 1; c <= B; ++c)
#pragma unroll
      for (int dk = 0; dk < B; ++dk) {
        const int j = i - c, kk = j + 1 + dk;
        Lv[c][dk] = (j >= 0 && kk < P) ? F[kk * WD + B - 1 - dk] : 0.0;
      }
    double ZR[WD];  // ZR[B + o] = Z(i, i + o)
#pragma unroll
    for (int c = B; c >= 0; --c) {
      double s = (c == 0) ? 1.0 : 0.0;
#pragma unroll
      for (int kk = 1; kk <= B; ++kk) s -= U[kk] * ZW[kk - 1][B + c - kk];
      ZR[B + c] = (i + c < P) ? s / U[0] : 0.0;
    }
#pragma unroll
    for (int c = 1; c <= B; ++c) {  // column j = i - c
      double s = 0.0;
#pragma unroll
      for (int dk = 0; dk < B; ++dk) s -= ZR[B - c + 1 + dk] * Lv[c][dk];
      ZR[B - c] = (i - c >= 0) ? s : 0.0;
    }
    for (int o = -r; o <= r; ++o)
      D[(size_t)i * (2 * r + 1) + (r + o)] = (i + o >= 0 && i + o < P) ? (R)ZR[B + o] : (R)0;
#pragma unroll
    for (int rr = B - 1; rr >= 1; --rr)
#pragma unroll
      for (int o = 0; o < WD; ++o) ZW[rr][o] = ZW[rr - 1][o];
#pragma unroll
    for (int o = 0; o < WD; ++o) ZW[0][o] = ZR[o];
  }
}

// ============================================================================ entropy
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_entropy_partial(const cplx<R>* __restrict__ img, size_t count,
                                                        double* __restrict__ partials) {
  double s = 0.0, tl = 0.0;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT) {
    const cplx<R> v = img[i];
    const R a = v.x * v.x + v.y * v.y;
    s += (double)a;
    if (a > (R)0) tl += (double)(a * log(a));
  }
  s = block_sum<NT>(s);
  tl = block_sum<NT>(tl);
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = s;
    partials[2 * blockIdx.x + 1] = tl;
  }
}

template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_entropy_finish(const cplx<R>* __restrict__ img, size_t count,
                                                       const double* __restrict__ partials, int nparts,
                                                       double* __restrict__ loss, cplx<R>* __restrict__ grad) {
  double s = 0.0, tl = 0.0;
  for (int i = threadIdx.x; i < nparts; i += NT) {
    s += partials[2 * i];
    tl += partials[2 * i + 1];
  }
  s = block_sum<NT>(s);
  tl = block_sum<NT>(tl);
  const double E = (s > 0.0) ? log(s) - tl / s : 0.0;  // E = ln S - (1/S) sum a ln a
  if (blockIdx.x == 0 && threadIdx.x == 0) *loss = E;
  if (!grad) return;
  const R logS = (R)log(s), Er = (R)E, sc = (R)(-2.0 / s);
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < count; i += (size_t)gridDim.x * NT) {
    const cplx<R> v = img[i];
    const R a = v.x * v.x + v.y * v.y;
    grad[i] = a > (R)0 ? (sc * (log(a) - logS + Er)) * v : cplx<R>{0, 0};
  }
}

// ============================================================================ debug FFT
template <typename R, int SIGN, int LOGN, int NT, int MAXRAD>
__global__ __launch_bounds__(NT) void k_fft(const cplx<R>* __restrict__ in, cplx<R>* out, const cplx<R>* __restrict__ tw) {
  constexpr int N = 1 << LOGN;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* twl = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = twl + tw_entries<N>();
  const size_t off = (size_t)blockIdx.x * N;
  load_twiddles<N, NT>(twl, tw);
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = in[off + i];
  __syncthreads();
  lds_fft<SIGN, N, NT, 1, MAXRAD, 1>(buf, twl);
  for (int i = threadIdx.x; i < N; i += NT) out[off + i] = buf[i];
}

// ============================================================================ launchers
template <int LOGN>
constexpr int nt_for() {
  return LOGN <= 8 ? 64 : (LOGN <= 11 ? 256 : (LOGN == 12 ? 256 : (LOGN == 13 ? 512 : 1024)));
}

int rows_threads(int logn) {
  switch (logn) {
    case 6: return nt_for<6>();
    case 7: return nt_for<7>();
    case 8: return nt_for<8>();
    case 9: return nt_for<9>();
    case 10: return nt_for<10>();
    case 11: return nt_for<11>();
    case 12: return nt_for<12>();
    case 13: return nt_for<13>();
    case 14: return nt_for<14>();
  }
  return 0;
}

static hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

size_t max_dynamic_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0)
    return (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    return (size_t)v;
  return 65536;
}

#define TFFR_LOGN_CASE(v, ...) \
  case v: {                     \
    constexpr int L = v;        \
    __VA_ARGS__                 \
  }
#define TFFR_LOGN_DISPATCH(logn, ...)     \
  switch (logn) {                         \
    TFFR_LOGN_CASE(6, __VA_ARGS__)        \
    TFFR_LOGN_CASE(7, __VA_ARGS__)        \
    TFFR_LOGN_CASE(8, __VA_ARGS__)        \
    TFFR_LOGN_CASE(9, __VA_ARGS__)        \
    TFFR_LOGN_CASE(10, __VA_ARGS__)       \
    TFFR_LOGN_CASE(11, __VA_ARGS__)       \
    TFFR_LOGN_CASE(12, __VA_ARGS__)       \
    TFFR_LOGN_CASE(13, __VA_ARGS__)       \
    TFFR_LOGN_CASE(14, __VA_ARGS__)       \
    default:                              \
      return hipErrorInvalidValue;        \
  }

template <int LOGN, int CB>
constexpr int nt_cols() {
  constexpr int want = ((1 << LOGN) / 8) * CB;
  return want < 64 ? 64 : (want > 1024 ? 1024 : want);
}

template <typename R>
hipError_t launch_fwd_rows(const Geo& g, const Tab<R>& t, int stype, const void* samples, const R* phase,
                           const R* dalong, const R* w, cplx<R>* out, int stage, hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfx) + ((size_t)1 << g.lognfx) / 64 + 64) +
                     sizeof(float) * kPolyLds;
  if (g.range_mode == 1 && g.W > kRunWindow) return hipErrorInvalidValue;
  TFFR_LOGN_DISPATCH(g.lognfx, {
    constexpr int NT = nt_for<L>();
    auto fn = g.range_mode == 1
                  ? k_fwd_rows_run<R, L, NT, kRunWindow>
                  : (g.sub <= 4 ? k_fwd_rows<R, L, NT, 4>
                                : (g.sub <= 8 ? k_fwd_rows<R, L, NT, 8> : k_fwd_rows<R, L, NT, 16>));
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(g.n_pulses), dim3(NT), lds, st, g, t, stype, samples, phase, dalong, w, out, stage);
    return hipGetLastError();
  })
}

#define TFFR_CB_DISPATCH(cb, ...)   \
  switch (cb) {                     \
    case 1: {                       \
      constexpr int CB = 1;         \
      __VA_ARGS__                   \
    }                               \
    case 2: {                       \
      constexpr int CB = 2;         \
      __VA_ARGS__                   \
    }                               \
    case 4: {                       \
      constexpr int CB = 4;         \
      __VA_ARGS__                   \
    }                               \
    default:                        \
      return hipErrorInvalidValue;  \
  }

template <typename R>
hipError_t launch_fwd_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* hx, cplx<R>* img, double* partials,
                           hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * ((((size_t)1 << g.lognfy) + g.n_pulses) * cb +
                                         ((size_t)1 << g.lognfy) / 64 + 64);
  const int grid = (g.mx + cb - 1) / cb;
  TFFR_LOGN_DISPATCH(g.lognfy, {
    TFFR_CB_DISPATCH(cb, {
      constexpr int NT = nt_cols<L, CB>();
      auto fn = k_fwd_cols<R, L, NT, CB>;
      hipError_t e = allow_lds((const void*)fn, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, st, g, t, hx, img, partials);
      return hipGetLastError();
    })
  })
}

template <typename R>
hipError_t launch_adj_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* cot, cplx<R>* hx, const double* stats,
                           const double* partials, int nparts, double* loss, hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfy) * cb + ((size_t)1 << g.lognfy) / 64 + 64);
  const int grid = (g.mx + cb - 1) / cb;
  TFFR_LOGN_DISPATCH(g.lognfy, {
    TFFR_CB_DISPATCH(cb, {
      constexpr int NT = nt_cols<L, CB>();
      auto fn = k_adj_cols<R, L, NT, CB>;
      hipError_t e = allow_lds((const void*)fn, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, st, g, t, cot, hx, stats, partials, nparts, loss);
      return hipGetLastError();
    })
  })
}

template <typename R>
hipError_t launch_ent_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* hx, cplx<R>* img, double* partials,
                           R* cblk, cplx<R>* h12, hipStream_t st) {
  const size_t nfy = (size_t)1 << g.lognfy;
  const size_t lds = sizeof(cplx<R>) * (nfy * cb + std::max<size_t>((size_t)g.n_pulses * cb, nfy * cb) + nfy / 64 + 64);
  const int grid = (g.mx + cb - 1) / cb;
  TFFR_LOGN_DISPATCH(g.lognfy, {
    TFFR_CB_DISPATCH(cb, {
      constexpr int NT = nt_cols<L, CB>();
      auto fn = k_ent_cols<R, L, NT, CB>;
      hipError_t e = allow_lds((const void*)fn, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, st, g, t, hx, img, partials, cblk, h12);
      return hipGetLastError();
    })
  })
}

template <typename R>
hipError_t launch_adj_rows(const Geo& g, const Tab<R>& t, int stype, const cplx<R>* hx, const void* samples,
                           const R* phase, const R* dalong, const R* w, cplx<R>* grad_s, R* grad_phase,
                           R* grad_dalong, const EntComb<R>& ec, hipStream_t st) {
  size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfx) + ((size_t)1 << g.lognfx) / 64 + 64) +
               sizeof(float) * kPolyLds;
  if (g.weighting == 2) lds += sizeof(cplx<R>) * (size_t)g.n_freq;
  TFFR_LOGN_DISPATCH(g.lognfx, {
    constexpr int NT = nt_for<L>();
    // short slices on a 2048-point row: twice the threads shorten the per-sample gather
    // (at most two samples per thread); longer slices keep the FFT's thread count
    constexpr int NT2 = L == 11 ? 512 : NT;
    const bool wide = NT2 != NT && g.n_freq <= 2 * NT2;
    auto fn = wide ? k_adj_rows<R, L, NT2> : k_adj_rows<R, L, NT>;
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(g.n_pulses), dim3(wide ? NT2 : NT), lds, st, g, t, stype, hx, samples, phase, dalong,
                       w, grad_s, grad_phase, grad_dalong, ec);
    return hipGetLastError();
  })
}

template <typename R>
static hipError_t launch_coord_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* cot, cplx<R>* h0,
                                   cplx<R>* h1, hipStream_t st) {
  const size_t nfy = (size_t)1 << g.lognfy;
  const size_t lds = sizeof(cplx<R>) * (2 * nfy * cb + nfy / 64 + 64);
  const int grid = (g.mx + cb - 1) / cb;
  TFFR_LOGN_DISPATCH(g.lognfy, {
    TFFR_CB_DISPATCH(cb, {
      constexpr int NT = nt_cols<L, CB>();
      auto fn = k_coord_cols<R, L, NT, CB>;
      hipError_t e = allow_lds((const void*)fn, lds);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(fn, dim3(grid), dim3(NT), lds, st, g, t, cot, h0, h1);
      return hipGetLastError();
    })
  })
}

template <typename R>
hipError_t launch_coord_grad(const Geo& g, const Tab<R>& t, int cb, int stype, const cplx<R>* cot, const void* samples,
                             const R* phase, const R* dalong, const R* w, cplx<R>* h0, cplx<R>* h1, R* grad_kx,
                             R* grad_ky, hipStream_t st) {
  hipError_t e = launch_coord_cols<R>(g, t, cb, cot, h0, h1, st);
  if (e != hipSuccess) return e;
  const size_t nfx = (size_t)1 << g.lognfx;
  const size_t lds = sizeof(cplx<R>) * (2 * nfx + nfx / 64 + 64) + sizeof(float) * kPolyLds;
  TFFR_LOGN_DISPATCH(g.lognfx, {
    constexpr int NT = nt_for<L>();
    auto fn = k_coord_rows<R, L, NT>;
    e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(g.n_pulses), dim3(NT), lds, st, g, t, stype, h0, h1, samples, phase, dalong, w,
                       grad_kx, grad_ky);
    return hipGetLastError();
  })
}

template <typename R>
hipError_t launch_row_phase_grad(const Geo& g, const Tab<R>& t, int stype, const void* samples, const cplx<R>* grad_s,
                                 R* grad_phase, R* grad_dalong, hipStream_t st) {
  hipLaunchKernelGGL((k_row_phase_grad<R, 256>), dim3(g.n_pulses), dim3(256), 0, st, g, t, stype, samples, grad_s,
                     grad_phase, grad_dalong);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_weights(const Geo& g, const Tab<R>& t, R* w, unsigned long long* kept_partial, int nblocks,
                          hipStream_t st) {
  hipLaunchKernelGGL((k_weights<R, 256>), dim3(nblocks), dim3(256), 0, st, g, t, w, kept_partial);
  return hipGetLastError();
}

hipError_t launch_entropy_stats(const double* partials, int nparts, double* stats, double* loss, hipStream_t st) {
  hipLaunchKernelGGL((k_entropy_stats<256>), dim3(1), dim3(256), 0, st, partials, nparts, stats, loss);
  return hipGetLastError();
}

hipError_t launch_sum_u64(const unsigned long long* parts, int n, long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(64), 0, st, parts, n, out);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_ffr(const Geo& g, const Tab<R>& t, double* scratch, R* dband, int* status, hipStream_t st) {
  // scratch: tap tables [N][2K+1] x 2, floors [N], band [N][2b+1]
  const size_t total = (size_t)g.n_pulses * g.n_freq;
  const int K = (int)ceil(g.q) + 1, KT = 2 * K + 1, WD = 2 * g.band_b + 1;
  double* tpsi = scratch;
  double* twt = tpsi + total * KT;
  double* gband = twt + total * KT;
  int* fl = reinterpret_cast<int*>(gband + total * WD);
  const int blocks = (int)std::min<size_t>((total + 255) / 256, 4096);
  hipLaunchKernelGGL((k_ffr_taps<R, 256>), dim3(blocks), dim3(256), 0, st, g, t, tpsi, twt, fl);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_ffr_build<R, 256>), dim3(blocks), dim3(256), 0, st, g, tpsi, twt, fl, gband);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds = sizeof(double) * (size_t)g.n_freq * WD;
  const dim3 grid(g.n_pulses), blk(64);
#define TFFR_FFR_SOLVE(BB)                                                                          \
  case BB: {                                                                                        \
    auto fn = k_ffr_solve<R, BB>;                                                                   \
    e = allow_lds((const void*)fn, lds);                                                            \
    if (e != hipSuccess) return e;                                                                  \
    hipLaunchKernelGGL(fn, grid, blk, lds, st, g, gband, dband, status);                            \
    break;                                                                                          \
  }
  switch (g.band_b) {
    TFFR_FFR_SOLVE(1)
    TFFR_FFR_SOLVE(2)
    TFFR_FFR_SOLVE(3)
    TFFR_FFR_SOLVE(4)
    TFFR_FFR_SOLVE(5)
    TFFR_FFR_SOLVE(6)
    default:
      return hipErrorInvalidValue;
  }
#undef TFFR_FFR_SOLVE
  return hipGetLastError();
}

template <typename R>
hipError_t launch_entropy(const Geo& g, const cplx<R>* img, double* partials, int nparts, double* loss,
                          cplx<R>* grad, hipStream_t st) {
  const size_t count = (size_t)g.mx * g.my;
  hipLaunchKernelGGL((k_entropy_partial<R, 256>), dim3(nparts), dim3(256), 0, st, img, count, partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int gblocks = grad ? nparts : 1;
  hipLaunchKernelGGL((k_entropy_finish<R, 256>), dim3(gblocks), dim3(256), 0, st, img, count, partials, nparts,
                     loss, grad);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_fft(int log2n, int batch, int sign, int max_radix, const cplx<R>* in, cplx<R>* out,
                      const cplx<R>* tw, hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * (((size_t)1 << log2n) + ((size_t)1 << log2n) / 64 + 64);
  TFFR_LOGN_DISPATCH(log2n, {
    constexpr int NT = nt_for<L>();
    auto fn = sign > 0 ? (max_radix == 16 ? k_fft<R, +1, L, NT, 16> : k_fft<R, +1, L, NT, 8>)
                       : (max_radix == 16 ? k_fft<R, -1, L, NT, 16> : k_fft<R, -1, L, NT, 8>);
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(batch), dim3(NT), lds, st, in, out, tw);
    return hipGetLastError();
  })
}

#define TFFR_INSTANTIATE(R)                                                                                     \
  template hipError_t launch_fwd_rows<R>(const Geo&, const Tab<R>&, int, const void*, const R*, const R*,     \
                                         const R*, cplx<R>*, int, hipStream_t);                                \
  template hipError_t launch_fwd_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, double*,     \
                                         hipStream_t);                                                         \
  template hipError_t launch_adj_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, const double*, \
                                         const double*, int, double*, hipStream_t);                             \
  template hipError_t launch_ent_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, double*, R*,   \
                                         cplx<R>*, hipStream_t);                                               \
  template hipError_t launch_adj_rows<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, const void*, const R*, \
                                         const R*, const R*, cplx<R>*, R*, R*, const EntComb<R>&, hipStream_t); \
  template hipError_t launch_coord_grad<R>(const Geo&, const Tab<R>&, int, int, const cplx<R>*, const void*,       \
                                           const R*, const R*, const R*, cplx<R>*, cplx<R>*, R*, R*, hipStream_t); \
  template hipError_t launch_row_phase_grad<R>(const Geo&, const Tab<R>&, int, const void*, const cplx<R>*, R*, R*, \
                                               hipStream_t);                                                  \
  template hipError_t launch_weights<R>(const Geo&, const Tab<R>&, R*, unsigned long long*, int, hipStream_t);  \
  template hipError_t launch_ffr<R>(const Geo&, const Tab<R>&, double*, R*, int*, hipStream_t);                \
  template hipError_t launch_entropy<R>(const Geo&, const cplx<R>*, double*, int, double*, cplx<R>*,          \
                                        hipStream_t);                                                          \
  template hipError_t launch_fft<R>(int, int, int, int, const cplx<R>*, cplx<R>*, const cplx<R>*, hipStream_t);

TFFR_INSTANTIATE(float)
TFFR_INSTANTIATE(double)

}  // namespace tffr
