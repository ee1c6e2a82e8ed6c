// Azimuth-stage kernels of libtffr: the forward azimuth gridding + FFT + deapodisation of
// CB range columns per workgroup (with the image-entropy partial sums on request), the
// reduction of those sums, and the type-2 azimuth adjoint (optionally forming the entropy
// gradient from the image).

#include "tffr_device.h"

namespace tffr {

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

// Image entropy from the per-block sums: E = ln S - (1/S) sum a ln a.  One block.
// stats[0] = S, stats[1] = E; *loss = E.  Each thread issues its (S, T) pair loads four
// at a time (one 16-byte load per pair), so the whole reduction waits on one or two
// memory latencies rather than one per pair.
template <int NT>
__global__ __launch_bounds__(NT) void k_entropy_stats(const double* __restrict__ partials, int nparts,
                                                      double* __restrict__ stats, double* __restrict__ loss) {
  constexpr int U = 4;
  const double2* pp = reinterpret_cast<const double2*>(partials);
  double s = 0.0, tl = 0.0;
  for (int i0 = threadIdx.x; i0 < nparts; i0 += U * NT) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      v[u] = i < nparts ? pp[i] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s += v[u].x;
      tl += v[u].y;
    }
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

// ============================================================================ launchers
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

#ifdef TFFR_EMIT_SHARED
hipError_t launch_entropy_stats(const double* partials, int nparts, double* stats, double* loss, hipStream_t st) {
  hipLaunchKernelGGL((k_entropy_stats<1024>), dim3(1), dim3(1024), 0, st, partials, nparts, stats, loss);
  return hipGetLastError();
}
#endif

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_fwd_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, double*, hipStream_t); \
  template hipError_t launch_adj_cols<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, cplx<R>*, const double*, const double*, int, double*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
