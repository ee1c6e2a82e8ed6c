// Range-migration front end (range FFT and matched filter; azimuth transform at uniform
// positions, or at positions with per-pulse errors) and
// Stolt-interpolation baseline of libtffr (Sec. II-A; Sec. IV, Baselines).
//
// Front end: raw echoes e[j][p] at J along-track positions u_j = (j - J/2) du become the
// samples s[n][p] = exp(+i kx(n,p) X_c) sum_j e[j][p] exp(-i ku_n u_j), ku_n = (n - N_u/2)
// 2 pi / (J du): with n' = n - N_u/2 the sum is (-1)^n' times bin n' mod J of the J-point
// forward DFT along azimuth.  CB fast-time columns per workgroup: the J x CB tile comes in
// as rows of CB contiguous values, is transformed in LDS (CB transforms back to back),
// and the centred N_u bins leave as rows of CB values after the reference multiply
// (phase kx X_c in FP64: it reaches 1e5 rad and more).
//
// Stolt: per azimuth slice, the samples are interpolated linearly onto the integer
// lattice l (kx = 2 pi l / fov_x) between the slice's first and last sample, and the
// range sum T[jx] = sum_l S(l) exp(2 pi i l X_jx / fov_x) is one inverse FFT of the fine
// row: with mx a power of two dividing the row length N, lattice point l sits exactly on
// cell l N / mx, and the readout at (jx - mx/2) mod N is that of the gridding kernels (no
// kernel, so no deapodisation).  Thread t takes the interval [lam_p, lam_{p+1}) of each of
// its samples and writes the lattice points inside it; the slice is cut into parts of
// samples spanning less than mx - 1 lattice units, so the points of one part fall on
// distinct cells (a plain read-add-write, one barrier per part).  The azimuth sum is the
// forward azimuth stage of the other methods.

#include <cstdlib>

#include "tffr_device.h"

namespace tffr {

// Two-level table of exp(+2 pi i m / N) (the layout of twiddle<N>) computed in FP64.
template <int N, int NT, typename R>
__device__ void make_twiddles(cplx<R>* tw) {
  for (int i = threadIdx.x; i < tw_entries<N>(); i += NT) {
    const int m = i < N / 64 ? 64 * i : i - N / 64;
    double s, c;
    sincospi(2.0 * (double)m / (double)N, &s, &c);
    tw[i] = {(R)c, (R)s};
  }
}

template <typename R, int LOGJ, int NT, int CB>
__global__ __launch_bounds__(NT) void k_rma_front(Geo g, Tab<R> t, const cplx<R>* __restrict__ echoes, double xc,
                                                  int stype, void* __restrict__ out) {
  constexpr int J = 1 << LOGJ;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<J>();  // [CB][J]
  const int P = g.n_freq, NU = g.n_pulses;
  const int p0 = xcd_block(blockIdx.x, gridDim.x) * CB;
  make_twiddles<J, NT>(tw);
  for (int idx = threadIdx.x; idx < J * CB; idx += NT) {
    const int j = idx / CB, c = idx - j * CB;
    buf[c * J + j] = p0 + c < P ? echoes[(size_t)j * P + p0 + c] : cplx<R>{0, 0};
  }
  __syncthreads();
  lds_fft<-1, J, NT, CB, 8, 2>(buf, tw);
  for (int idx = threadIdx.x; idx < NU * CB; idx += NT) {
    const int n = idx / CB, c = idx - n * CB, p = p0 + c;
    if (p >= P) continue;
    const int nn = n - NU / 2;
    cplx<R> v = buf[c * J + (nn & (J - 1))];
    if (nn & 1) v = {-v.x, -v.y};
    double sn, cs;
    sincos(stolt_kx(t.k[p], t.ku[n]) * xc, &sn, &cs);
    v = cmul(v, cplx<R>{(R)cs, (R)sn});
    const size_t o = (size_t)n * P + p;
    if (stype == ST_H2) {
      ((half2s*)out)[o] = {(_Float16)(float)v.x, (_Float16)(float)v.y};
    } else {
      ((cplx<R>*)out)[o] = v;
    }
  }
}

// Range FFT and matched filter: pulse j's P baseband time samples -> its centred frequency
// bins E[j][p] = ref[p] sum_t r[j][t] exp(-2 pi i (p - P/2) t / P) (ref null: ones), the
// fast-time samples the front end takes.  One pulse per workgroup, transformed in LDS; a
// workgroup reads its whole row before writing it, so the output may alias the input.
template <typename R, int LOGP, int NT>
__global__ __launch_bounds__(NT) void k_rma_range_fft(const cplx<R>* pulses, const cplx<R>* __restrict__ ref,
                                                      cplx<R>* echoes) {
  constexpr int P = 1 << LOGP;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<P>();
  const size_t row = (size_t)blockIdx.x * P;
  make_twiddles<P, NT>(tw);
  for (int i = threadIdx.x; i < P; i += NT) buf[i] = pulses[row + i];
  __syncthreads();
  lds_fft<-1, P, NT, 1, 8, 1>(buf, tw);
  for (int p = threadIdx.x; p < P; p += NT) {
    cplx<R> v = buf[(p - P / 2) & (P - 1)];
    if (ref) v = cmul(v, ref[p]);
    echoes[row + p] = v;
  }
}

// Front end with per-pulse position errors: echo j was recorded at u_j + d_j, so the
// azimuth sum s[n] = sum_j e[j] exp(-i ku_n (u_j + d_j)) = sum_j e[j] exp(-2 pi i n' t_j),
// t_j = (u_j + d_j) / (J du), is a type-1 NUFFT at the non-uniform t_j: the echoes are
// spread with the ES kernel onto a periodic grid of G cells at g_j = G t_j (pos[j]), the
// grid is transformed forward, and bin n' is divided by the kernel's transform (deapf).
// A workgroup takes CB fast-time columns; sources are spread in S sub-passes, sub-pass
// sp taking j = sp, sp + S, ...: S is a power of two (it divides J) with S times the
// smallest gap between consecutive positions (cyclically) above W + 1 cells, so the taps
// of one sub-pass never meet and each is a plain read-add-write followed by a barrier.
template <typename R, int LOGG, int NT, int CB>
__global__ __launch_bounds__(NT) void k_rma_front_pos(Geo g, Tab<R> t, const cplx<R>* __restrict__ echoes,
                                                      const double* __restrict__ pos, int J, int S, double xc,
                                                      int stype, void* __restrict__ out) {
  constexpr int G = 1 << LOGG;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<G>();  // [CB][G]
  const int P = g.n_freq, NU = g.n_pulses, W = g.W;
  const int p0 = xcd_block(blockIdx.x, gridDim.x) * CB;
  const R halfw = (R)(0.5 * W), inv_halfw = (R)(2.0 / W), beta = es_shape<R>(g);
  make_twiddles<G, NT>(tw);
  for (int i = threadIdx.x; i < CB * G; i += NT) buf[i] = {0, 0};
  __syncthreads();
  for (int sp = 0; sp < S; ++sp) {
    for (int j = sp + S * (int)threadIdx.x; j < J; j += S * NT) {
      cplx<R> e[CB];
#pragma unroll
      for (int c = 0; c < CB; ++c) e[c] = p0 + c < P ? echoes[(size_t)j * P + p0 + c] : cplx<R>{0, 0};
      const double gj = pos[j];
      const double fl = floor(gj);
      const R f = (R)(gj - fl);
      const int k0 = (int)ceil(f - halfw);
      const int cell = (int)fl + k0;
      const R z0 = ((R)k0 - f) * inv_halfw;
      for (int i = 0; i < W; ++i) {
        const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
        const int q = (cell + i) & (G - 1);
#pragma unroll
        for (int c = 0; c < CB; ++c) buf[c * G + q] = buf[c * G + q] + phi * e[c];
      }
    }
    __syncthreads();
  }
  lds_fft<-1, G, NT, CB, 8, 2>(buf, tw);
  for (int idx = threadIdx.x; idx < NU * CB; idx += NT) {
    const int n = idx / CB, c = idx - n * CB, p = p0 + c;
    if (p >= P) continue;
    const int nn = n - NU / 2;
    cplx<R> v = t.deapf[n] * buf[c * G + (nn & (G - 1))];
    double sn, cs;
    sincos(stolt_kx(t.k[p], t.ku[n]) * xc, &sn, &cs);
    v = cmul(v, cplx<R>{(R)cs, (R)sn});
    const size_t o = (size_t)n * P + p;
    if (stype == ST_H2) {
      ((half2s*)out)[o] = {(_Float16)(float)v.x, (_Float16)(float)v.y};
    } else {
      ((cplx<R>*)out)[o] = v;
    }
  }
}

template <typename R, int LOGN, int NT>
__global__ __launch_bounds__(NT) void k_stolt_rows(Geo g, Tab<R> t, int stype, const void* __restrict__ samples,
                                                   const R* __restrict__ phase, const R* __restrict__ dalong,
                                                   int part, cplx<R>* __restrict__ out) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = (N + NT - 1) / NT;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();
  const int n = blockIdx.x, P = g.n_freq, mx = g.mx;
  const int step = N / mx;  // fine cells per lattice unit
  const size_t base = (size_t)n * P;
  load_twiddles<N, NT>(tw, t.twx);
  for (int i = threadIdx.x; i < N; i += NT) buf[i] = {0, 0};
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  __syncthreads();
  for (int pa = 0; pa < P; pa += part) {
    const int pb = min(pa + part, P);
    for (int p = pa + (int)threadIdx.x; p < pb; p += NT) {
      const double la = lattice_coord(kx_of(t, raw_k(t, P, n, p), ku), g);
      const bool last = p + 1 == P;
      const double lb = last ? la : lattice_coord(kx_of(t, raw_k(t, P, n, p + 1), ku), g);
      const cplx<R> sa = load_sample<R>(samples, stype, base + p);
      const cplx<R> sb = last ? sa : load_sample<R>(samples, stype, base + p + 1);
      const double inv = last ? 0.0 : 1.0 / (lb - la);
      // lattice points l with la <= l < lb (and l = la at the slice's last sample)
      for (double l = ceil(la); l < lb || (last && l == la); l += 1.0) {
        const R tt = (R)((l - la) * inv);
        const cplx<R> v = cmul(rot, sa + tt * (sb - sa));
        const long long li = (long long)l;
        const int cell = (int)(((li % mx) + mx) % mx) * step;
        buf[cell] = buf[cell] + v;
        if (last) break;
      }
    }
    __syncthreads();
  }
  lds_fft<+1, N, NT, 1, 8, 1>(buf, tw);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    if (jx < mx) out[(size_t)n * mx + jx] = buf[(jx - mx / 2) & (N - 1)];
  }
}

// ============================================================================ launchers
template <typename R>
hipError_t launch_rma_front(const Geo& g, const Tab<R>& t, int logj, const cplx<R>* echoes, double xc, int stype,
                            void* out, hipStream_t st) {
  const int J = 1 << logj;
  // columns per workgroup: the widest of 16, 8, 4, 2, 1 whose J x CB tile fits 128 KB of
  // LDS and still gives 512 workgroups (two per CU); wider tiles read longer runs of each
  // echo row, narrower ones fill the chip
  const size_t col = (size_t)J * sizeof(cplx<R>);
  int cb = 0;
  for (int c = 16; c >= 1; c /= 2) {
    if ((size_t)c * col > ((size_t)128 << 10)) continue;
    cb = c;
    if ((g.n_freq + c - 1) / c >= 512) break;
  }
  if (const char* ev = std::getenv("TFFR_RMA_CB")) {  // tuning: force a width that fits
    const int f = std::atoi(ev);
    if ((f == 1 || f == 2 || f == 4 || f == 8 || f == 16) && (size_t)f * col <= ((size_t)128 << 10)) cb = f;
  }
  if (cb == 0) return hipErrorInvalidValue;
  const size_t lds = sizeof(cplx<R>) * ((size_t)J / 64 + 64) + (size_t)cb * col;
  const int nblk = (g.n_freq + cb - 1) / cb;
#define TFFR_RMA_CB(CBV)                                                                  \
  if (cb == CBV) {                                                                        \
    constexpr int NT = nt_cols<L, CBV>();                                                 \
    auto fn = k_rma_front<R, L, NT, CBV>;                                                 \
    hipError_t e = allow_lds((const void*)fn, lds);                                       \
    if (e != hipSuccess) return e;                                                        \
    hipLaunchKernelGGL(fn, dim3(nblk), dim3(NT), lds, st, g, t, echoes, xc, stype, out);  \
    return hipGetLastError();                                                             \
  }
  TFFR_LOGN_DISPATCH(logj, {
    TFFR_RMA_CB(16)
    TFFR_RMA_CB(8)
    TFFR_RMA_CB(4)
    TFFR_RMA_CB(2)
    TFFR_RMA_CB(1)
    return hipErrorInvalidValue;
  })
#undef TFFR_RMA_CB
}

template <typename R>
hipError_t launch_rma_range_fft(int logp, int n_rows, const cplx<R>* pulses, const cplx<R>* ref, cplx<R>* echoes,
                                hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * (((size_t)1 << logp) + ((size_t)1 << logp) / 64 + 64);
  TFFR_LOGN_DISPATCH(logp, {
    constexpr int NT = nt_for<L>();
    auto fn = k_rma_range_fft<R, L, NT>;
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(n_rows), dim3(NT), lds, st, pulses, ref, echoes);
    return hipGetLastError();
  })
}

template <typename R>
hipError_t launch_rma_front_pos(const Geo& g, const Tab<R>& t, int logg, const cplx<R>* echoes, const double* pos,
                                int J, int S, double xc, int stype, void* out, hipStream_t st) {
  const int G = 1 << logg;
  // columns per workgroup as for the uniform front end: the widest of 16 ... 1 whose
  // G x CB row fits 128 KB of LDS and still gives 512 workgroups
  const size_t col = (size_t)G * sizeof(cplx<R>);
  int cb = 0;
  for (int c = 16; c >= 1; c /= 2) {
    if ((size_t)c * col > ((size_t)128 << 10)) continue;
    cb = c;
    if ((g.n_freq + c - 1) / c >= 512) break;
  }
  if (cb == 0 || S < 1) return hipErrorInvalidValue;
  const size_t lds = sizeof(cplx<R>) * ((size_t)G / 64 + 64) + (size_t)cb * col;
  const int nblk = (g.n_freq + cb - 1) / cb;
#define TFFR_RMA_POS_CB(CBV)                                                                         \
  if (cb == CBV) {                                                                                 \
    constexpr int NT = nt_cols<L, CBV>();                                                          \
    auto fn = k_rma_front_pos<R, L, NT, CBV>;                                                      \
    hipError_t e = allow_lds((const void*)fn, lds);                                                \
    if (e != hipSuccess) return e;                                                                 \
    hipLaunchKernelGGL(fn, dim3(nblk), dim3(NT), lds, st, g, t, echoes, pos, J, S, xc, stype, out); \
    return hipGetLastError();                                                                      \
  }
  TFFR_LOGN_DISPATCH(logg, {
    TFFR_RMA_POS_CB(16)
    TFFR_RMA_POS_CB(8)
    TFFR_RMA_POS_CB(4)
    TFFR_RMA_POS_CB(2)
    TFFR_RMA_POS_CB(1)
    return hipErrorInvalidValue;
  })
#undef TFFR_RMA_POS_CB
}

template <typename R>
hipError_t launch_stolt_rows(const Geo& g, const Tab<R>& t, int stype, const void* samples, const R* phase,
                             const R* dalong, int part, cplx<R>* out, hipStream_t st) {
  const size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfx) + ((size_t)1 << g.lognfx) / 64 + 64);
  if (part < 1 || ((1 << g.lognfx) % g.mx) != 0) return hipErrorInvalidValue;
  TFFR_LOGN_DISPATCH(g.lognfx, {
    constexpr int NT = nt_for<L>();
    auto fn = k_stolt_rows<R, L, NT>;
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(g.n_pulses), dim3(NT), lds, st, g, t, stype, samples, phase, dalong, part, out);
    return hipGetLastError();
  })
}

#define TFFR_INSTANTIATE(R)                                                                                      \
  template hipError_t launch_rma_front<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, double, int, void*,    \
                                          hipStream_t);                                                          \
  template hipError_t launch_stolt_rows<R>(const Geo&, const Tab<R>&, int, const void*, const R*, const R*, int, \
                                           cplx<R>*, hipStream_t);                                             \
  template hipError_t launch_rma_range_fft<R>(int, int, const cplx<R>*, const cplx<R>*, cplx<R>*, hipStream_t);   \
  template hipError_t launch_rma_front_pos<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, const double*, int, \
                                              int, double, int, void*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
