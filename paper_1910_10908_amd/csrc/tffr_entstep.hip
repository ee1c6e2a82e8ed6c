// Fused entropy-step azimuth kernel of libtffr: per column block, the image columns, their
// share of the entropy sums, and the adjoint azimuth transforms of the two fields the
// entropy gradient is linear in.

#include "tffr_device.h"

namespace tffr {

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

// ============================================================================ launchers
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

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_ent_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, double*, R*, cplx<R>*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
