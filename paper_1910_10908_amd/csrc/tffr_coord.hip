// Coordinate-gradient kernels of libtffr: dL/dkx per sample and dL/dky per slice for an
// image cotangent (azimuth stage over two fields, then the range stage).

#include "tffr_device.h"

namespace tffr {

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
    bool kept;
    const cplx<R> c =
        weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lattice_coord(kx, g), rot, sp, kept);
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

// ============================================================================ launchers
template <typename R>
hipError_t launch_coord_cols(const Geo& g, const Tab<R>& t, int cb, const cplx<R>* cot, cplx<R>* h0,
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

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_coord_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, cplx<R>*, hipStream_t); \
  template hipError_t launch_coord_grad<R>(const Geo&, const Tab<R>&, int, int, const cplx<R>*, const void*, const R*, const R*, const R*, cplx<R>*, cplx<R>*, R*, R*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
