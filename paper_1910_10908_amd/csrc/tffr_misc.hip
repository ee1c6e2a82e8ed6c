// Auxiliary kernels of libtffr: materialised weights and the kept count, the standalone
// image entropy, the per-slice phase-gradient reduction and the single-FFT test hook.

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
  template hipError_t launch_entropy<R>(const Geo&, const cplx<R>*, double*, int, double*, cplx<R>*, hipStream_t); \
  template hipError_t launch_fft<R>(int, int, int, int, const cplx<R>*, cplx<R>*, const cplx<R>*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
