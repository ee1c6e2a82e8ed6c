// Device-side building blocks shared by the kernel sources of libtffr (gfx950, CDNA4):
// complex arithmetic, XCD-aware block numbering, reductions, the LDS Stockham FFT,
// coordinate reduction, the method's weights, the ES gridding kernel, the azimuth
// stage's gather / interpolation helpers, and the launch-configuration helpers.
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

#pragma once

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

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }
// Radix of the stage after spans P: MAXRAD while it fits, then what is left.  With
// MAXRAD 8, radix-16 first stages take the place of a small last stage: one where
// log2 N = 1 mod 3 (16, 128, 1024, 8192: 16 8 8 8 instead of 8 8 8 8 2), and in single
// precision two where log2 N = 2 mod 3 from 256 points up (2048: 16 16 8 instead of
// 8 8 8 4; in double precision the second radix-16 stage's registers cost more).
template <int N, int P, int MAXRAD, int RB>
constexpr int stage_radix() {
  constexpr int lg = ilog2c(N);
  if constexpr (MAXRAD == 8 && P == 1 && lg % 3 == 1 && lg >= 4) return 16;
  if constexpr (MAXRAD == 8 && RB == 4 && (P == 1 || P == 16) && lg % 3 == 2 && lg >= 8) return 16;
  return (N / P) >= MAXRAD ? MAXRAD : (N / P);
}

template <int SIGN, int N, int P, int NT, int NBAT, int MAXRAD, int SWZ, typename R>
__device__ __forceinline__ void fft_from(cplx<R>* buf, const cplx<R>* tw) {
  if constexpr (P < N) {
    constexpr int RB = (int)sizeof(R);
    constexpr int RAD = stage_radix<N, P, MAXRAD, RB>();
    constexpr bool in = P > 1 && (SWZ == 1 || (SWZ == 2 && P == stage_radix<N, 1, MAXRAD, RB>()));
    constexpr bool out = P * RAD < N && (SWZ == 1 || (SWZ == 2 && P == 1));
    fft_stage<SIGN, N, RAD, P, NT, NBAT, in, out>(buf, tw);
    fft_from<SIGN, N, P * RAD, NT, NBAT, MAXRAD, SWZ>(buf, tw);
  }
}

// out[j] = sum_g buf[g] exp(SIGN 2 pi i g j / N) for NBAT transforms stored back to back
// in LDS, in place, natural order; tw is the LDS twiddle table.  Call with all NT
// threads after a barrier.
// Stages of radix MAXRAD (8 or 16) and one smaller last stage (with MAXRAD 8, one or two
// radix-16 first stages where that removes the small last stage: see stage_radix).  Radix 16 takes fewer LDS
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
static __device__ double frame_diag(double delta, double a, double q, double ema2, double epa2) {
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
static __device__ __attribute__((noinline)) double tffr_weight_f64(double delta, double a, double q, double ema2,
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
    // the same predicates as the FP64 path: literal |1/g| >= tau; correlation g >= tau,
    // i.e. 1/g > 0 and 1/g <= 1/tau (thr_f holds tau or 1/tau)
    const float thr = g.thr_f;
    if (g.thresh_mode == 0) {
      const float av = fabsf(v);
      if (fabsf(av - thr) > g.near_f * thr) return av >= thr ? (R)v : (R)0;
    } else {
      if (!(v > 0.0f)) return (R)0;
      if (fabsf(v - thr) > g.near_f * thr) return v <= thr ? (R)v : (R)0;
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
static __device__ __forceinline__ double lit_tap(double d, double sgn, double s0, double c0, double a, double ema2) {
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
// `kept` is false when a diagonal weight is zero (a sample the threshold removes, Sec.
// III-C): the caller then skips its taps.
template <typename R>
__device__ __forceinline__ cplx<R> weighted_sample(const Geo& g, const Tab<R>& t, const float* poly, int stype,
                                                   const void* samples, const R* w, int n, int p,
                                                   double ku, double lam, cplx<R> rot, cplx<R> s, bool& kept) {
  const size_t base = (size_t)n * g.n_freq;
  kept = true;
  if (g.weighting == 2)  // plain FFR: banded D within the slice
    return cmul(rot, ffr_apply<R>(samples, stype, w, base, p, g.n_freq, g.band_r));
  const R wt = w ? w[base + p] : diag_weight<R>(g, t, poly, ku, n, p, lam);
  kept = wt != (R)0;
  return wt * cmul(rot, s);
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

// ----------------------------------------------------------------------------- launch configuration
template <int LOGN>
constexpr int nt_for() {
  return LOGN <= 8 ? 64 : (LOGN <= 11 ? 256 : (LOGN == 12 ? 256 : (LOGN == 13 ? 512 : 1024)));
}

static inline hipError_t allow_lds(const void* fn, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

// Each kernel source instantiates its launchers for one compute type per object when the
// build defines TFFR_REAL_F32 or TFFR_REAL_F64 (the two objects compile in parallel), and
// for both otherwise.  Code that is not per type goes into one object only
// (TFFR_EMIT_SHARED).
#if defined(TFFR_REAL_F32)
#define TFFR_INSTANTIATE_TYPES TFFR_INSTANTIATE(float)
#elif defined(TFFR_REAL_F64)
#define TFFR_INSTANTIATE_TYPES TFFR_INSTANTIATE(double)
#else
#define TFFR_INSTANTIATE_TYPES \
  TFFR_INSTANTIATE(float)      \
  TFFR_INSTANTIATE(double)
#endif
#if !defined(TFFR_REAL_F64)
#define TFFR_EMIT_SHARED 1
#endif

}  // namespace tffr
