// Auxiliary kernels of libtffr: materialised weights and the kept count, the plain-FFR
// banded solve, the standalone image entropy, the per-slice phase-gradient reduction and
// the single-FFT test hook.

#include "tffr_device.h"

namespace tffr {

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

#ifdef TFFR_EMIT_SHARED
__global__ void k_sum_u64(const unsigned long long* __restrict__ parts, int n, long long* out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    unsigned long long s = 0;
    for (int i = 0; i < n; ++i) s += parts[i];
    *out = (long long)s;
  }
}
#endif

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
#ifdef TFFR_EMIT_SHARED
size_t max_dynamic_lds() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeSharedMemPerBlockOptin, dev) == hipSuccess && v > 0)
    return (size_t)v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && v > 0)
    return (size_t)v;
  return 65536;
}
#endif

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

#ifdef TFFR_EMIT_SHARED
hipError_t launch_sum_u64(const unsigned long long* parts, int n, long long* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_u64, dim3(1), dim3(64), 0, st, parts, n, out);
  return hipGetLastError();
}
#endif

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
    TFFR_FFR_SOLVE(7)
    TFFR_FFR_SOLVE(8)
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

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_row_phase_grad<R>(const Geo&, const Tab<R>&, int, const void*, const cplx<R>*, R*, R*, hipStream_t); \
  template hipError_t launch_weights<R>(const Geo&, const Tab<R>&, R*, unsigned long long*, int, hipStream_t); \
  template hipError_t launch_ffr<R>(const Geo&, const Tab<R>&, double*, R*, int*, hipStream_t); \
  template hipError_t launch_entropy<R>(const Geo&, const cplx<R>*, double*, int, double*, cplx<R>*, hipStream_t); \
  template hipError_t launch_fft<R>(int, int, int, int, const cplx<R>*, cplx<R>*, const cplx<R>*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
