// Range-stage kernels of libtffr: type-1 gridding of each azimuth slice with the fused
// coordinate prep and weights (sub-pass and run variants), and the type-2
// range adjoint with the per-slice phase / position gradient reduction.

#include "tffr_device.h"

namespace tffr {

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
              bool kept;
              const cplx<R> c = weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lam, rot, sr[j], kept);
              if (!kept) {
                // removed by the threshold: no taps
              } else if (g.literal) {
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

// Range stage, run variant (the plan's choice for non-literal gridding with W <= WM).
// Thread t takes the run of S consecutive samples p0 = part start + S t ... and
// read-add-writes each sample's W taps straight into the LDS row.  The lanes of a wave
// step through their runs together, and samples S apart are more than W cells apart
// (the plan picks S with S * (smallest sample spacing) > W + 1), so no two lanes touch a
// cell in the same step; a wave's LDS operations complete in issue order, so a cell two
// lanes reach in different steps is updated in turn.  Runs only meet their neighbours'
// cells, and only the first run of each wave (lane 0) has its neighbour in another wave:
// that lane sends the taps of its samples that start within W cells of its run's first
// cell to a halo of its own, added to the row after the part's barrier.  Taps that run
// past the row end land in a pad of PAD cells, folded onto the row start before the FFT.
// The WW taps of one sample read-add-written at dst[0, WW): the cells are read back to
// back, the kernel values formed meanwhile, then the sums written.
template <int WW, typename R>
__device__ __forceinline__ void run_taps(cplx<R>* dst, R z0, R dz, R beta, cplx<R> c) {
  cplx<R> v[WW];
#pragma unroll
  for (int i = 0; i < WW; ++i) v[i] = dst[i];
#pragma unroll
  for (int i = 0; i < WW; ++i) dst[i] = v[i] + es_kernel(z0 + (R)i * dz, beta) * c;
}

// The taps of two consecutive samples whose first cells are c0 and c0 + d1 (d1 0 or 1),
// summed in registers and read-add-written once over the WW + 1 cells from c0.
template <int WW, typename R>
__device__ __forceinline__ void run_taps_pair(cplx<R>* dst, R za, R zb, bool d1, R dz, R beta, cplx<R> ca,
                                              cplx<R> cb) {
  cplx<R> v[WW + 1];
#pragma unroll
  for (int i = 0; i <= WW; ++i) v[i] = dst[i];
  R pa[WW], pb[WW];
#pragma unroll
  for (int i = 0; i < WW; ++i) {
    pa[i] = es_kernel(za + (R)i * dz, beta);
    pb[i] = es_kernel(zb + (R)i * dz, beta);
  }
#pragma unroll
  for (int k = 0; k <= WW; ++k) {
    const R ta = k < WW ? pa[k] : (R)0;
    const R tb = d1 ? (k >= 1 ? pb[k - 1] : (R)0) : (k < WW ? pb[k] : (R)0);
    dst[k] = v[k] + ta * ca + tb * cb;
  }
}

// sum_i phi_i dst[i] over the WW taps of one sample: the cells are read back to back.
template <int WW, typename R>
__device__ __forceinline__ cplx<R> gather_taps(const cplx<R>* src, R z0, R dz, R beta) {
  cplx<R> v[WW];
#pragma unroll
  for (int i = 0; i < WW; ++i) v[i] = src[i];
  cplx<R> a = {0, 0};
#pragma unroll
  for (int i = 0; i < WW; ++i) a = a + es_kernel(z0 + (R)i * dz, beta) * v[i];
  return a;
}

// waves per SIMD the paired run kernel's registers are sized for (complex64): the
// workgroups per CU its LDS row allows (160 KB per CU), at most four waves
template <typename R, int LOGN, int NT, bool PAIR>
constexpr int run_waves() {
  if constexpr (sizeof(R) != 4 || !PAIR) {
    return 1;
  } else {
    constexpr int wg = (160 * 1024) / ((int)sizeof(cplx<R>) * ((1 << LOGN) + 512) + 4096);
    constexpr int w = (wg < 1 ? 1 : wg) * (NT / 64) / 4;
    return w < 1 ? 1 : (w > 4 ? 4 : w);
  }
}

template <typename R, int LOGN, int NT, int WM, bool PAIR, int QP>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(run_waves<R, LOGN, NT, PAIR>())))
void k_fwd_rows_run(Geo g, Tab<R> t, int stype, const void* __restrict__ samples,
                                                     const R* __restrict__ phase, const R* __restrict__ dalong,
                                                     const R* __restrict__ w, cplx<R>* __restrict__ out,
                                                     int stage) {
  constexpr int N = 1 << LOGN;
  constexpr int DPT = (N + NT - 1) / NT;
  constexpr int NW = NT / 64;
  constexpr int PAD = 2 * WM;
  constexpr int LPP = NT / QP;  // lanes per part in flight
  static_assert(QP == 1 || (QP == 2 && LPP % 64 == 0), "parts in flight");
  static_assert(NW <= kRunHaloInts, "one halo start per wave");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();  // [QP][N + PAD]: one row per part in flight
  cplx<R>* halo = buf + QP * (N + PAD);  // [NW][PAD]
  int* hcf = reinterpret_cast<int*>(halo + NW * PAD);  // [NW] halo's first cell (-1: none)
  float* lpoly = reinterpret_cast<float*>(hcf + kRunHaloInts);
  const int n = blockIdx.x;
  const bool ffr = g.weighting == 2;
  const int S = g.sub, W = g.W, plen = g.part_len;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const size_t base_s = (size_t)n * g.n_freq;
  load_twiddles<N, NT>(tw, t.twx);
  const float* poly = load_poly<NT>(g, t.poly, lpoly);
  for (int i = threadIdx.x; i < QP * (N + PAD) + NW * PAD; i += NT) buf[i] = {0, 0};
  // with QP = 2 the first half of the threads takes one part and the second half the next
  // one, each in its own row (a slice's parts overlap once wrapped onto the row)
  const int q = QP == 1 ? 0 : (int)threadIdx.x / LPP;
  const int tq = (int)threadIdx.x - q * LPP;
  cplx<R>* row = buf + q * (N + PAD);
  const cplx<R> rot = row_rotation(t, phase, dalong, n);
  const double ku = t.ku[n];
  const R halfw = (R)(0.5 * g.W), inv_halfw = (R)(2.0 / g.W), beta = es_shape<R>(g);
  __syncthreads();  // row zeroed, tables in LDS
  for (int pg = 0; pg < g.n_freq; pg += QP * plen) {
    const int pa = pg + q * plen;
    const int pb = min(pa + plen, g.n_freq);
    const int p0 = pa + S * tq;
    const int p1 = min(p0 + S, pb);
    int cfirst = 0;
    // one sample's weighted value, first tap cell (unwrapped: only differences and the low
    // LOGN bits are used), kernel offset and fraction; false if the threshold removed it
    auto prep = [&](int p, double kp, cplx<R> sp, int& c0, int& k0, R& f, cplx<R>& c) {
      const double kx = kx_of(t, kp, ku);
      const double lam = lattice_coord(kx, g);
      bool kept;
      c = weighted_sample<R>(g, t, poly, stype, samples, w, n, p, ku, lam, rot, sp, kept);
      const double tt = kx * g.tx_scale;
      int ui;
      fine_pos<R>(tt, N, ui, f);
      k0 = (int)ceil(f - halfw);
      c0 = (int)((unsigned)(int)floor(tt) * (unsigned)N + (unsigned)(ui + k0));
      return kept;
    };
    auto single = [&](int c0, int k0, R f, cplx<R> c) {
      const int rel = c0 - cfirst;
      cplx<R>* dst = (lane == 0 && rel < W) ? halo + wv * PAD + rel : row + (c0 & (N - 1));
      const R z0 = ((R)k0 - f) * inv_halfw;
      switch (W) {  // uniform: one unrolled tap block per kernel width
#define TFFR_RUN_TAPS(WW) \
  case WW: run_taps<WW>(dst, z0, inv_halfw, beta, c); break;
        TFFR_RUN_TAPS(2)
        TFFR_RUN_TAPS(3)
        TFFR_RUN_TAPS(4)
        TFFR_RUN_TAPS(5)
        TFFR_RUN_TAPS(6)
        TFFR_RUN_TAPS(7)
        TFFR_RUN_TAPS(8)
#undef TFFR_RUN_TAPS
      }
    };
    if constexpr (!PAIR) {
      double k_nx = p0 < p1 ? raw_k(t, g.n_freq, n, p0) : 0.0;
      cplx<R> s_nx = (p0 < p1 && !ffr) ? load_sample<R>(samples, stype, base_s + p0) : cplx<R>{0, 0};
      for (int p = p0; p < p1; ++p) {
        const double kp = k_nx;
        const cplx<R> sp = s_nx;
        if (p + 1 < p1) {
          k_nx = raw_k(t, g.n_freq, n, p + 1);
          if (!ffr) s_nx = load_sample<R>(samples, stype, base_s + p + 1);
        }
        int c0, k0;
        R f;
        cplx<R> c;
        const bool kept = prep(p, kp, sp, c0, k0, f, c);
        if (p == p0) cfirst = c0;
        if (kept) single(c0, k0, f, c);  // a removed sample has no taps
      }
    } else {
      // samples two at a time (the plan's S keeps samples S - 1 apart more than W cells
      // apart, so the two samples of every lane in a step stay clear of the other lanes')
      double ka = 0.0, kb = 0.0;
      cplx<R> sa = {0, 0}, sb = {0, 0};
      if (p0 < p1) {
        ka = raw_k(t, g.n_freq, n, p0);
        if (!ffr) sa = load_sample<R>(samples, stype, base_s + p0);
      }
      if (p0 + 1 < p1) {
        kb = raw_k(t, g.n_freq, n, p0 + 1);
        if (!ffr) sb = load_sample<R>(samples, stype, base_s + p0 + 1);
      }
      for (int p = p0; p < p1; p += 2) {
        const double kpa = ka, kpb = kb;
        const cplx<R> spa = sa, spb = sb;
        if (p + 2 < p1) {
          ka = raw_k(t, g.n_freq, n, p + 2);
          if (!ffr) sa = load_sample<R>(samples, stype, base_s + p + 2);
        }
        if (p + 3 < p1) {
          kb = raw_k(t, g.n_freq, n, p + 3);
          if (!ffr) sb = load_sample<R>(samples, stype, base_s + p + 3);
        }
        int c0a, k0a;
        R fa;
        cplx<R> ca;
        const bool kept_a = prep(p, kpa, spa, c0a, k0a, fa, ca);
        if (p == p0) cfirst = c0a;
        const bool has_b = p + 1 < p1;
        int c0b = c0a, k0b = 0;
        R fb = 0;
        cplx<R> cb = {0, 0};
        bool kept_b = false;
        if (has_b) kept_b = prep(p + 1, kpb, spb, c0b, k0b, fb, cb);
        const int d = c0b - c0a;
        if (W == 7 && has_b && (d == 0 || d == 1) && (kept_a || kept_b)) {
          // removed samples carry a zero value here
          const int rel = c0a - cfirst;
          cplx<R>* dst = (lane == 0 && rel < W) ? halo + wv * PAD + rel : row + (c0a & (N - 1));
          run_taps_pair<7>(dst, ((R)k0a - fa) * inv_halfw, ((R)k0b - fb) * inv_halfw, d == 1, inv_halfw, beta,
                           kept_a ? ca : cplx<R>{0, 0}, kept_b ? cb : cplx<R>{0, 0});
        } else {
          if (kept_a) single(c0a, k0a, fa, ca);
          if (kept_b) single(c0b, k0b, fb, cb);
        }
      }
    }
    if (lane == 0) hcf[wv] = p0 < p1 ? q * (N + PAD) + (cfirst & (N - 1)) : -1;
    __syncthreads();
    // halos onto the row: distinct waves' halos hold distinct cells of the part
    for (int i = threadIdx.x; i < NW * PAD; i += NT) {
      const int hw = i / PAD, j = i - hw * PAD;
      const int cf = hcf[hw];
      if (cf >= 0) {
        cplx<R>& bb = buf[cf + j];
        bb = bb + halo[i];
      }
      halo[i] = cplx<R>{0, 0};
    }
    __syncthreads();
  }
  if constexpr (QP == 2) {  // the second row onto the first
    for (int i = threadIdx.x; i < N + PAD; i += NT) buf[i] = buf[i] + buf[N + PAD + i];
    __syncthreads();
  }
  // the pad onto the row start
  if (threadIdx.x < PAD) buf[threadIdx.x] = buf[threadIdx.x] + buf[N + threadIdx.x];
  __syncthreads();
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
  // radix 16 (fewer LDS passes); 8192 single-precision points as 16 8 8 8 rather than
  // 16 16 16 2
  lds_fft<+1, N, NT, 1, (LOGN == 13 && sizeof(R) == 4 ? 8 : 16), 1>(buf, tw);
#pragma unroll
  for (int j = 0; j < DPT; ++j) {
    const int jx = threadIdx.x + j * NT;
    if (jx < mx) out[(size_t)n * mx + jx] = dx[j] * buf[(jx - mx / 2) & (N - 1)];
  }
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
  constexpr int PAD = 2 * kRunWindow;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem);
  cplx<R>* buf = tw + tw_entries<N>();  // [N + PAD]: the row, then a copy of its first PAD cells
  float* lpoly = reinterpret_cast<float*>(buf + N + PAD);
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
  // the row's first cells once more past its end, so a sample's taps are W consecutive cells
  if (threadIdx.x < PAD) buf[N + threadIdx.x] = buf[threadIdx.x];
  __syncthreads();
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
    // diagonal weight first: a sample the threshold removes needs no gather
    const R wt = ffr ? (R)1 : (w ? wp : diag_weight<R>(g, t, poly, ku, n, p, lattice_coord(kx, g)));
    cplx<R> a = {0, 0};
    if (wt == (R)0) {
      // removed by the threshold: zero gradient
    } else if (g.literal) {
      a = lit_gather<R>(buf, N, kx * g.tx_scale, g.q, g.lit_taps, g.a, g.ema2);
    } else {
      int ui;
      R f;
      fine_pos<R>(kx * g.tx_scale, N, ui, f);
      const int k0 = (int)ceil(f - halfw);
      const cplx<R>* src = buf + ((ui + k0) & (N - 1));
      const R z0 = ((R)k0 - f) * inv_halfw;
      if (g.W <= kRunWindow) {
        switch (g.W) {  // uniform: one unrolled tap block per kernel width
#define TFFR_ADJ_TAPS(WW) \
  case WW: a = gather_taps<WW>(src, z0, inv_halfw, beta); break;
          TFFR_ADJ_TAPS(2)
          TFFR_ADJ_TAPS(3)
          TFFR_ADJ_TAPS(4)
          TFFR_ADJ_TAPS(5)
          TFFR_ADJ_TAPS(6)
          TFFR_ADJ_TAPS(7)
          TFFR_ADJ_TAPS(8)
#undef TFFR_ADJ_TAPS
        }
      } else {
        const int cell = ui + k0;
        for (int i = 0; i < g.W; ++i) {
          const R phi = es_kernel(z0 + (R)i * inv_halfw, beta);
          a = a + phi * buf[(cell + i) & (N - 1)];
        }
      }
    }
    if (ffr) {
      gbuf[p] = a;
      continue;
    }
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

// ============================================================================ launchers
// the run kernel, paired (complex64 rows of 4096 cells and more, the plan's choice for
// samples under half a cell apart) or one sample at a time
template <typename R, int L, int NT>
static auto run_kernel(bool pair, bool two_parts) {
  if constexpr (sizeof(R) == 4 && L >= 12) {
    if (pair) return k_fwd_rows_run<R, L, NT, kRunWindow, true, 1>;
  }
  if constexpr (L <= 12 && 2 * NT <= 1024 && 2 * NT / 64 <= kRunHaloInts) {
    if (two_parts) return k_fwd_rows_run<R, L, 2 * NT, kRunWindow, false, 2>;
  }
  return k_fwd_rows_run<R, L, NT, kRunWindow, false, 1>;
}

#ifdef TFFR_EMIT_SHARED
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
#endif

template <typename R>
hipError_t launch_fwd_rows(const Geo& g, const Tab<R>& t, int stype, const void* samples, const R* phase,
                           const R* dalong, const R* w, cplx<R>* out, int stage, hipStream_t st) {
  size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfx) + ((size_t)1 << g.lognfx) / 64 + 64) +
               sizeof(float) * kPolyLds;
  if (g.range_mode == 1 && g.W > kRunWindow) return hipErrorInvalidValue;
  TFFR_LOGN_DISPATCH(g.lognfx, {
    constexpr int NT = nt_for<L>();
    static_assert(NT / 64 <= kRunHaloInts, "run kernel halos");
    // run kernel: the row's pad and one halo per wave, 2 kRunWindow cells each; with two
    // parts at once a second row with its pad, on twice the threads
    constexpr bool can_two = L <= 12 && 2 * NT <= 1024 && 2 * NT / 64 <= kRunHaloInts;
    const bool two = can_two && g.range_mode == 1 && g.run_parts == 2 && !g.run_pair;
    const int nt = two ? 2 * NT : NT;
    if (g.range_mode == 1) {
      lds += sizeof(cplx<R>) * (size_t)(2 * kRunWindow) * (1 + nt / 64) + sizeof(int) * kRunHaloInts;
      if (two) lds += sizeof(cplx<R>) * (((size_t)1 << L) + 2 * kRunWindow);
    }
    auto fn = g.range_mode == 1
                  ? run_kernel<R, L, NT>(g.run_pair != 0, two)
                  : (g.sub <= 4 ? k_fwd_rows<R, L, NT, 4>
                                : (g.sub <= 8 ? k_fwd_rows<R, L, NT, 8> : k_fwd_rows<R, L, NT, 16>));
    hipError_t e = allow_lds((const void*)fn, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(fn, dim3(g.n_pulses), dim3(nt), lds, st, g, t, stype, samples, phase, dalong, w, out, stage);
    return hipGetLastError();
  })
}

template <typename R>
hipError_t launch_adj_rows(const Geo& g, const Tab<R>& t, int stype, const cplx<R>* hx, const void* samples,
                           const R* phase, const R* dalong, const R* w, cplx<R>* grad_s, R* grad_phase,
                           R* grad_dalong, const EntComb<R>& ec, hipStream_t st) {
  size_t lds = sizeof(cplx<R>) * (((size_t)1 << g.lognfx) + 2 * kRunWindow + ((size_t)1 << g.lognfx) / 64 + 64) +
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

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_fwd_rows<R>(const Geo&, const Tab<R>&, int, const void*, const R*, const R*, const R*, cplx<R>*, int, hipStream_t); \
  template hipError_t launch_adj_rows<R>(const Geo&, const Tab<R>&, int, const cplx<R>*, const void*, const R*, const R*, const R*, cplx<R>*, R*, R*, const EntComb<R>&, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
