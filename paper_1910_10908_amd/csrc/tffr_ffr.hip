// Plain-FFR weights of libtffr: D = B_r(pinv(Psi W)) per azimuth slice (Eq. (8); band
// B_r, r = 2 in Sec. IV).  The truncated frame product of a slice factors over the lattice
// points the slice reaches, G~ = A B^T with A[p][l] = R_Psi(l - lam_p) and B[p][l] =
// R_W(l - lam_p) (|l - lam_p| < q; G~ carries R_Psi on the row sample, R_W on the column
// sample), and G~ is banded in the sample index.  Two routes, one workgroup per slice:
//
//  * full rank (samples more than a lattice unit apart): the band of G~ itself, then the
//    band of its inverse by block cyclic reduction (selected inversion);
//  * rank deficient (more samples than lattice points, A and B of full column rank):
//    pinv(A B^T) = B (B^T B)^-1 (A^T A)^-1 A^T, so D[p][p'] = sum_{l,l'} B[p][l] N[l][l']
//    A[p'][l'] with N = (Sa Sb)^-1, Sa = A^T A and Sb = B^T B banded Gram matrices of the
//    lattice points; the band of N again by block cyclic reduction.
//
// Block cyclic reduction on a matrix of half-band HB, cut into blocks of HB rows (block
// tridiagonal): at level s the nodes that are odd multiples of s are eliminated in
// parallel (their Schur complements update the even neighbours, which become neighbours
// at distance 2s), down to node 0; the selected inverse then comes back up the levels,
// each eliminated node taking Z of its diagonal block and of its two couplings from the
// already known Z of its neighbours (Z_ia = -X_a Z_aa - X_b Z_ba etc. with
// X = D_i^-1 A_i.).  Every entry of the inverse within the blocks' band is produced: the
// diagonal blocks and the couplings of adjacent blocks.  FP64 throughout.  The status word
// receives the worst outcome over the slices: 1 a block pivot below 1e-13 of the matrix
// scale, 3 an inverse whose band reaches 1e15 over the matrix scale (no correct digit
// left; on the rank-deficient route both measured after diagonal equilibration), 2 a
// slice reaching more lattice points than the plan provided for.

#include "tffr_device.h"

namespace tffr {

constexpr int kFfrMaxKT = 11;  // lattice taps per sample: 2 (ceil(q) + 1) + 1 for q <= 4

// R_Psi and R_W at the lattice points m = floor(lam) + k, k in [-K, K]; zero where
// |m - lam| >= q.  One sincospi(delta) serves every tap: sin(pi (k - delta)) =
// -(-1)^k sin(pi delta), cos(pi (k - delta)) = (-1)^k cos(pi delta).
__device__ __forceinline__ void frame_taps(double lam, const Geo& g, int K, double* rp, double* rw, int& fl) {
  const double f = floor(lam), delta = lam - f;
  fl = (int)f;
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
    rp[k + K] = vp;
    rw[k + K] = vw;
  }
}

// ---------------------------------------------------------------- small dense blocks
// B x B row-major blocks in the workgroup's scratch (global memory, cache resident); the
// products keep one row or column of B values in registers.  Every block argument of one
// call is a different block (the reduction never passes a block as both operand and
// result), which the restrict qualifiers state: the loads of a call need not wait for its
// stores.
template <int B>
__device__ void mm(double* __restrict__ C, const double* __restrict__ X, const double* __restrict__ Y) {  // C = X Y
  for (int i = 0; i < B; ++i) {
    double row[B];
#pragma unroll
    for (int j = 0; j < B; ++j) row[j] = 0.0;
    for (int k = 0; k < B; ++k) {
      const double x = X[i * B + k];
#pragma unroll
      for (int j = 0; j < B; ++j) row[j] += x * Y[k * B + j];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) C[i * B + j] = row[j];
  }
}
template <int B>
__device__ void mm_acc(double* __restrict__ C, double sgn, const double* __restrict__ X,
                       const double* __restrict__ Y) {  // C += sgn X Y
  for (int i = 0; i < B; ++i) {
    double row[B];
#pragma unroll
    for (int j = 0; j < B; ++j) row[j] = 0.0;
    for (int k = 0; k < B; ++k) {
      const double x = X[i * B + k];
#pragma unroll
      for (int j = 0; j < B; ++j) row[j] += x * Y[k * B + j];
    }
#pragma unroll
    for (int j = 0; j < B; ++j) C[i * B + j] += sgn * row[j];
  }
}
template <int B>
__device__ void left_mul_inplace(const double* __restrict__ X, double* __restrict__ Y) {  // Y = X Y, column by column
  for (int j = 0; j < B; ++j) {
    double col[B];
#pragma unroll
    for (int k = 0; k < B; ++k) col[k] = Y[k * B + j];
    for (int i = 0; i < B; ++i) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) s += X[i * B + k] * col[k];
      Y[i * B + j] = s;
    }
  }
}
template <int B>
__device__ void right_mul_inplace(double* __restrict__ Y, const double* __restrict__ X) {  // Y = Y X, row by row
  for (int i = 0; i < B; ++i) {
    double row[B];
#pragma unroll
    for (int k = 0; k < B; ++k) row[k] = Y[i * B + k];
    for (int j = 0; j < B; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) s += row[k] * X[k * B + j];
      Y[i * B + j] = s;
    }
  }
}
// M = M^-1 by Gauss-Jordan elimination with partial pivoting on [M | T] (T: a spare
// block, left holding the inverse, then copied back; blocks of up to 5 x 5 are eliminated
// in registers instead); false when a pivot falls below tol.
template <int B>
__device__ bool inv_block(double* __restrict__ M, double* __restrict__ T, double tol) {
  if constexpr (B <= 5) {  // small blocks: the whole elimination in registers
    double a[B][B], t[B][B];
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int j = 0; j < B; ++j) {
        a[i][j] = M[i * B + j];
        t[i][j] = i == j ? 1.0 : 0.0;
      }
#pragma unroll
    for (int c = 0; c < B; ++c) {
      int piv = c;
      double best = fabs(a[c][c]);
#pragma unroll
      for (int r = c + 1; r < B; ++r)
        if (fabs(a[r][c]) > best) {
          best = fabs(a[r][c]);
          piv = r;
        }
      if (!(best > tol)) return false;
#pragma unroll
      for (int r = c + 1; r < B; ++r)
        if (piv == r)
#pragma unroll
          for (int j = 0; j < B; ++j) {
            double u = a[c][j];
            a[c][j] = a[r][j];
            a[r][j] = u;
            u = t[c][j];
            t[c][j] = t[r][j];
            t[r][j] = u;
          }
      const double inv = 1.0 / a[c][c];
#pragma unroll
      for (int j = 0; j < B; ++j) {
        a[c][j] *= inv;
        t[c][j] *= inv;
      }
#pragma unroll
      for (int r = 0; r < B; ++r)
        if (r != c) {
          const double l = a[r][c];
#pragma unroll
          for (int j = 0; j < B; ++j) {
            a[r][j] -= l * a[c][j];
            t[r][j] -= l * t[c][j];
          }
        }
    }
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int j = 0; j < B; ++j) M[i * B + j] = t[i][j];
    return true;
  }
  for (int i = 0; i < B; ++i)
    for (int j = 0; j < B; ++j) T[i * B + j] = i == j ? 1.0 : 0.0;
  for (int c = 0; c < B; ++c) {
    int piv = c;
    for (int r = c + 1; r < B; ++r)
      if (fabs(M[r * B + c]) > fabs(M[piv * B + c])) piv = r;
    if (!(fabs(M[piv * B + c]) > tol)) return false;
    if (piv != c)
      for (int j = 0; j < B; ++j) {
        double t = M[c * B + j];
        M[c * B + j] = M[piv * B + j];
        M[piv * B + j] = t;
        t = T[c * B + j];
        T[c * B + j] = T[piv * B + j];
        T[piv * B + j] = t;
      }
    const double inv = 1.0 / M[c * B + c];
    for (int j = 0; j < B; ++j) {
      M[c * B + j] *= inv;
      T[c * B + j] *= inv;
    }
    for (int r = 0; r < B; ++r)
      if (r != c) {
        const double l = M[r * B + c];
        if (l != 0.0)
          for (int j = 0; j < B; ++j) {
            M[r * B + j] -= l * M[c * B + j];
            T[r * B + j] -= l * T[c * B + j];
          }
      }
  }
  for (int e = 0; e < B * B; ++e) M[e] = T[e];
  return true;
}

// Register-held B x B blocks (small B): a task loads every operand block it needs at once,
// computes, and stores its results, one memory round trip instead of one per product.
template <int B>
struct Blk {
  double v[B][B];
};
template <int B>
__device__ __forceinline__ Blk<B> ldb(const double* p) {
  Blk<B> b;
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) b.v[i][j] = p[i * B + j];
  return b;
}
template <int B>
__device__ __forceinline__ void stb(double* p, const Blk<B>& b, double sgn = 1.0) {
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) p[i * B + j] = sgn * b.v[i][j];
}
template <int B>
__device__ __forceinline__ Blk<B> zerob() {
  Blk<B> b;
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) b.v[i][j] = 0.0;
  return b;
}
template <int B>
__device__ __forceinline__ void macb(Blk<B>& c, double sgn, const Blk<B>& x, const Blk<B>& y) {  // c += sgn x y
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) {
      double acc = 0.0;
#pragma unroll
      for (int k = 0; k < B; ++k) acc += x.v[i][k] * y.v[k][j];
      c.v[i][j] += sgn * acc;
    }
}
template <int B>
__device__ __forceinline__ Blk<B> mulb(const Blk<B>& x, const Blk<B>& y) {
  Blk<B> c = zerob<B>();
  macb<B>(c, 1.0, x, y);
  return c;
}
// a = a^-1 by Gauss-Jordan with partial pivoting; false when a pivot falls below tol
template <int B>
__device__ __forceinline__ bool invb(Blk<B>& a, double tol) {
  Blk<B> t;
#pragma unroll
  for (int i = 0; i < B; ++i)
#pragma unroll
    for (int j = 0; j < B; ++j) t.v[i][j] = i == j ? 1.0 : 0.0;
  bool ok = true;
#pragma unroll
  for (int c = 0; c < B; ++c) {
    int piv = c;
    double best = fabs(a.v[c][c]);
#pragma unroll
    for (int r = c + 1; r < B; ++r)
      if (fabs(a.v[r][c]) > best) {
        best = fabs(a.v[r][c]);
        piv = r;
      }
    if (!(best > tol)) ok = false;
#pragma unroll
    for (int r = c + 1; r < B; ++r)
      if (piv == r)
#pragma unroll
        for (int j = 0; j < B; ++j) {
          double u = a.v[c][j];
          a.v[c][j] = a.v[r][j];
          a.v[r][j] = u;
          u = t.v[c][j];
          t.v[c][j] = t.v[r][j];
          t.v[r][j] = u;
        }
    const double inv = ok ? 1.0 / a.v[c][c] : 0.0;
#pragma unroll
    for (int j = 0; j < B; ++j) {
      a.v[c][j] *= inv;
      t.v[c][j] *= inv;
    }
#pragma unroll
    for (int r = 0; r < B; ++r)
      if (r != c) {
        const double l = a.v[r][c];
#pragma unroll
        for (int j = 0; j < B; ++j) {
          a.v[r][j] -= l * a.v[c][j];
          t.v[r][j] -= l * t.v[c][j];
        }
      }
  }
  a = t;
  return ok;
}

// Selected inversion of one banded n x n matrix (half-band <= HB) by block cyclic
// reduction, by the NT threads of a workgroup.  band [n][2HB+1] (entry (i, j) at
// i (2HB+1) + HB + j - i) in; zband the same layout out (every entry within the band);
// work: 10 nb HB^2 doubles, nb = ceil(n / HB).  Returns false (all threads) when a block
// pivot vanishes.
template <int HB, int NT>
__device__ bool band_selinv(int n, const double* band, double* work, double* zband, double tol) {
  constexpr int BB = HB * HB, WD = 2 * HB + 1;
  __shared__ int bad;
  const int nb = (n + HB - 1) / HB;
  double* Dm = work;            // diagonal blocks (Schur complements), then their inverses
  double* Lm = Dm + nb * BB;    // coupling to the current left neighbour; X_a once eliminated
  double* Um = Lm + nb * BB;    // coupling to the current right neighbour; X_b once eliminated
  double* Ra = Um + nb * BB;    // A_{a,i}: the left neighbour's coupling to node i when i is eliminated
  double* Rb = Ra + nb * BB;    // A_{b,i}
  double* Zd = Rb + nb * BB;    // Z_ii (spare block of the inversion before that)
  double* ZL = Zd + nb * BB;    // Z_{i,a}
  double* ZLt = ZL + nb * BB;   // Z_{a,i}
  double* ZR = ZLt + nb * BB;   // Z_{i,b}
  double* ZRt = ZR + nb * BB;   // Z_{b,i}
  if (threadIdx.x == 0) bad = 0;
  auto entry = [&](int i, int j) -> double {  // padded rows / columns: identity
    if (i >= n || j >= n) return (i == j) ? 1.0 : 0.0;
    if (j < 0 || j - i > HB || i - j > HB) return 0.0;
    return band[(size_t)i * WD + HB + (j - i)];
  };
  for (int idx = threadIdx.x; idx < nb * BB; idx += NT) {
    const int bi = idx / BB, e = idx - bi * BB, r = e / HB, c = e - r * HB;
    const int row = bi * HB + r;
    Dm[idx] = entry(row, bi * HB + c);
    Um[idx] = (bi + 1 < nb) ? entry(row, (bi + 1) * HB + c) : 0.0;
    Lm[idx] = (bi > 0) ? entry(row, (bi - 1) * HB + c) : 0.0;
  }
  __syncthreads();
  int top = 1;
  while (top < nb) top *= 2;
  if constexpr (HB <= 5) {
    // Small blocks: every task holds its operand blocks in registers (one batch of loads,
    // the products, one batch of stores); the independent products of a node are tasks
    // q = 0..3 of it, on threads 4k + q.
    using BK = Blk<HB>;
    for (int s = 1; s < nb; s *= 2) {
      // eliminated nodes i (odd multiples of s): D_i^-1, X_a = D_i^-1 A_ia, X_b = D_i^-1 A_ib
      // (task 0), and the neighbours' couplings to i (task 1)
      for (int w = threadIdx.x;; w += NT) {
        const int k = w >> 2, q = w & 3;
        const int i = s * (2 * k + 1);
        if (i >= nb) break;
        const int a = i - s, b = i + s;
        if (q == 0) {
          BK d = ldb<HB>(Dm + (size_t)i * BB);
          const BK l = ldb<HB>(Lm + (size_t)i * BB), u = ldb<HB>(Um + (size_t)i * BB);
          if (!invb<HB>(d, tol)) bad = 1;
          stb<HB>(Dm + (size_t)i * BB, d);
          stb<HB>(Lm + (size_t)i * BB, mulb<HB>(d, l));
          stb<HB>(Um + (size_t)i * BB, mulb<HB>(d, u));
        } else if (q == 1) {
          const BK ra = ldb<HB>(Um + (size_t)a * BB);
          const BK rb = b < nb ? ldb<HB>(Lm + (size_t)b * BB) : zerob<HB>();
          stb<HB>(Ra + (size_t)i * BB, ra);
          stb<HB>(Rb + (size_t)i * BB, rb);
        }
      }
      __syncthreads();
      // surviving nodes j (multiples of 2s): Schur complement of both eliminated neighbours
      // (task 0), new couplings at distance 2s (tasks 1 and 2)
      for (int w = threadIdx.x;; w += NT) {
        const int k = w >> 2, q = w & 3;
        const int j = 2 * s * k;
        if (j >= nb) break;
        const int il = j - s, ir = j + s;
        if (q == 0) {
          BK d = ldb<HB>(Dm + (size_t)j * BB);
          const BK rbl = il >= 0 ? ldb<HB>(Rb + (size_t)il * BB) : zerob<HB>();
          const BK xbl = il >= 0 ? ldb<HB>(Um + (size_t)il * BB) : zerob<HB>();
          const BK rar = ir < nb ? ldb<HB>(Ra + (size_t)ir * BB) : zerob<HB>();
          const BK xar = ir < nb ? ldb<HB>(Lm + (size_t)ir * BB) : zerob<HB>();
          macb<HB>(d, -1.0, rbl, xbl);  // A_{j,il} X_b(il)
          macb<HB>(d, -1.0, rar, xar);  // A_{j,ir} X_a(ir)
          stb<HB>(Dm + (size_t)j * BB, d);
        } else if (q == 1) {  // A'_{j, j-2s} = -A_{j,il} X_a(il)
          const BK lj = il >= 0 ? mulb<HB>(ldb<HB>(Rb + (size_t)il * BB), ldb<HB>(Lm + (size_t)il * BB)) : zerob<HB>();
          stb<HB>(Lm + (size_t)j * BB, lj, -1.0);
        } else if (q == 2) {  // A'_{j, j+2s} = -A_{j,ir} X_b(ir)
          const BK uj = ir < nb ? mulb<HB>(ldb<HB>(Ra + (size_t)ir * BB), ldb<HB>(Um + (size_t)ir * BB)) : zerob<HB>();
          stb<HB>(Um + (size_t)j * BB, uj, -1.0);
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {  // the root (node 0): its Schur complement inverted
      BK d = ldb<HB>(Dm);
      if (!invb<HB>(d, tol)) bad = 1;
      stb<HB>(Dm, d);
      stb<HB>(Zd, d);
    }
    __syncthreads();
    for (int s = top / 2; s >= 1; s /= 2) {
      // the four couplings of Z of each node eliminated at level s
      for (int w = threadIdx.x;; w += NT) {
        const int k = w >> 2, q = w & 3;
        const int i = s * (2 * k + 1);
        if (i >= nb) break;
        const int a = i - s, b = i + s;
        const bool hb = b < nb;
        const double* pab = nullptr;
        const double* pba = nullptr;
        if (hb) {
          if ((a / (2 * s)) & 1) {
            pab = ZR + (size_t)a * BB;
            pba = ZRt + (size_t)a * BB;
          } else {
            pab = ZLt + (size_t)b * BB;
            pba = ZL + (size_t)b * BB;
          }
        }
        if (q == 0) {  // Z_{i,a} = -(X_a Z_aa + X_b Z_ba)
          const BK xa = ldb<HB>(Lm + (size_t)i * BB), zaa = ldb<HB>(Zd + (size_t)a * BB);
          const BK xb = hb ? ldb<HB>(Um + (size_t)i * BB) : zerob<HB>();
          const BK zba = hb ? ldb<HB>(pba) : zerob<HB>();
          BK z = mulb<HB>(xa, zaa);
          macb<HB>(z, 1.0, xb, zba);
          stb<HB>(ZL + (size_t)i * BB, z, -1.0);
        } else if (q == 1) {  // Z_{i,b} = -(X_a Z_ab + X_b Z_bb)
          BK z = zerob<HB>();
          if (hb) {
            const BK xa = ldb<HB>(Lm + (size_t)i * BB), zab = ldb<HB>(pab);
            const BK xb = ldb<HB>(Um + (size_t)i * BB), zbb = ldb<HB>(Zd + (size_t)b * BB);
            z = mulb<HB>(xa, zab);
            macb<HB>(z, 1.0, xb, zbb);
          }
          stb<HB>(ZR + (size_t)i * BB, z, -1.0);
        } else if (q == 2) {  // Z_{a,i} = -(Z_aa A_{a,i} + Z_ab A_{b,i}) D_i^-1
          const BK zaa = ldb<HB>(Zd + (size_t)a * BB), ra = ldb<HB>(Ra + (size_t)i * BB);
          const BK zab = hb ? ldb<HB>(pab) : zerob<HB>();
          const BK rb = hb ? ldb<HB>(Rb + (size_t)i * BB) : zerob<HB>();
          const BK di = ldb<HB>(Dm + (size_t)i * BB);
          BK z = mulb<HB>(zaa, ra);
          macb<HB>(z, 1.0, zab, rb);
          stb<HB>(ZLt + (size_t)i * BB, mulb<HB>(z, di), -1.0);
        } else {  // Z_{b,i} = -(Z_ba A_{a,i} + Z_bb A_{b,i}) D_i^-1
          BK z = zerob<HB>();
          if (hb) {
            const BK zba = ldb<HB>(pba), ra = ldb<HB>(Ra + (size_t)i * BB);
            const BK zbb = ldb<HB>(Zd + (size_t)b * BB), rb = ldb<HB>(Rb + (size_t)i * BB);
            const BK di = ldb<HB>(Dm + (size_t)i * BB);
            BK y = mulb<HB>(zba, ra);
            macb<HB>(y, 1.0, zbb, rb);
            z = mulb<HB>(y, di);
          }
          stb<HB>(ZRt + (size_t)i * BB, z, -1.0);
        }
      }
      __syncthreads();
      // Z_ii = D_i^-1 - X_a Z_{a,i} - X_b Z_{b,i}
      for (int k = threadIdx.x;; k += NT) {
        const int i = s * (2 * k + 1);
        if (i >= nb) break;
        const bool hb = i + s < nb;
        BK z = ldb<HB>(Dm + (size_t)i * BB);
        const BK xa = ldb<HB>(Lm + (size_t)i * BB), zlt = ldb<HB>(ZLt + (size_t)i * BB);
        const BK xb = hb ? ldb<HB>(Um + (size_t)i * BB) : zerob<HB>();
        const BK zrt = hb ? ldb<HB>(ZRt + (size_t)i * BB) : zerob<HB>();
        macb<HB>(z, -1.0, xa, zlt);
        macb<HB>(z, -1.0, xb, zrt);
        stb<HB>(Zd + (size_t)i * BB, z);
      }
      __syncthreads();
    }
  } else {
    // ---- elimination, level by level
    for (int s = 1; s < nb; s *= 2) {
      // phase 1: eliminated nodes i (odd multiples of s): D_i^-1, X_a = D_i^-1 A_ia,
      // X_b = D_i^-1 A_ib, and the neighbours' couplings to i
      for (int k = threadIdx.x;; k += NT) {
        const int i = s * (2 * k + 1);
        if (i >= nb) break;
        const int a = i - s, b = i + s;
        double* Di = Dm + (size_t)i * BB;
        if (!inv_block<HB>(Di, Zd + (size_t)i * BB, tol)) bad = 1;
        left_mul_inplace<HB>(Di, Lm + (size_t)i * BB);  // X_a
        left_mul_inplace<HB>(Di, Um + (size_t)i * BB);  // X_b (zero when i has no right neighbour)
        for (int e = 0; e < BB; ++e) Ra[(size_t)i * BB + e] = Um[(size_t)a * BB + e];
        for (int e = 0; e < BB; ++e) Rb[(size_t)i * BB + e] = b < nb ? Lm[(size_t)b * BB + e] : 0.0;
      }
      __syncthreads();
      // phase 2: surviving nodes j (multiples of 2s) take the Schur complement of both
      // eliminated neighbours and their new couplings at distance 2s
      for (int k = threadIdx.x;; k += NT) {
        const int j = 2 * s * k;
        if (j >= nb) break;
        const int il = j - s, ir = j + s;
        double* Dj = Dm + (size_t)j * BB;
        if (il >= 0) mm_acc<HB>(Dj, -1.0, Rb + (size_t)il * BB, Um + (size_t)il * BB);  // A_{j,il} X_b(il)
        if (ir < nb) mm_acc<HB>(Dj, -1.0, Ra + (size_t)ir * BB, Lm + (size_t)ir * BB);  // A_{j,ir} X_a(ir)
        double* Lj = Lm + (size_t)j * BB;
        double* Uj = Um + (size_t)j * BB;
        if (il >= 0) {  // A'_{j, j-2s} = -A_{j,il} X_a(il)
          mm<HB>(Lj, Rb + (size_t)il * BB, Lm + (size_t)il * BB);
          for (int e = 0; e < BB; ++e) Lj[e] = -Lj[e];
        } else {
          for (int e = 0; e < BB; ++e) Lj[e] = 0.0;
        }
        if (ir < nb) {  // A'_{j, j+2s} = -A_{j,ir} X_b(ir)
          mm<HB>(Uj, Ra + (size_t)ir * BB, Um + (size_t)ir * BB);
          for (int e = 0; e < BB; ++e) Uj[e] = -Uj[e];
        } else {
          for (int e = 0; e < BB; ++e) Uj[e] = 0.0;
        }
      }
      __syncthreads();
    }
    // ---- the root (node 0): its Schur complement inverted
    if (threadIdx.x == 0) {
      if (!inv_block<HB>(Dm, ZL, tol)) bad = 1;
      for (int e = 0; e < BB; ++e) Zd[e] = Dm[e];
    }
    __syncthreads();
    // ---- selected inversion back up the levels
    for (int s = top / 2; s >= 1; s /= 2) {
      for (int k = threadIdx.x;; k += NT) {
        const int i = s * (2 * k + 1);
        if (i >= nb) break;
        const int a = i - s, b = i + s;
        const bool hb = b < nb;
        const double* Xa = Lm + (size_t)i * BB;
        const double* Xb = Um + (size_t)i * BB;
        const double* Di = Dm + (size_t)i * BB;
        const double* Zaa = Zd + (size_t)a * BB;
        const double* Zbb = Zd + (size_t)(hb ? b : a) * BB;
        // Z_ab, Z_ba: a and b are neighbours at level 2s; the odd multiple of 2s among them
        // was eliminated there and holds the pair
        const double* Zab = nullptr;
        const double* Zba = nullptr;
        if (hb) {
          if ((a / (2 * s)) & 1) {
            Zab = ZR + (size_t)a * BB;
            Zba = ZRt + (size_t)a * BB;
          } else {
            Zab = ZLt + (size_t)b * BB;
            Zba = ZL + (size_t)b * BB;
          }
        }
        double* zl = ZL + (size_t)i * BB;
        double* zr = ZR + (size_t)i * BB;
        double* zlt = ZLt + (size_t)i * BB;
        double* zrt = ZRt + (size_t)i * BB;
        // Z_{i,a} = -(X_a Z_aa + X_b Z_ba), Z_{i,b} = -(X_a Z_ab + X_b Z_bb)
        mm<HB>(zl, Xa, Zaa);
        if (hb) mm_acc<HB>(zl, 1.0, Xb, Zba);
        for (int e = 0; e < BB; ++e) zl[e] = -zl[e];
        if (hb) {
          mm<HB>(zr, Xa, Zab);
          mm_acc<HB>(zr, 1.0, Xb, Zbb);
          for (int e = 0; e < BB; ++e) zr[e] = -zr[e];
        } else {
          for (int e = 0; e < BB; ++e) zr[e] = 0.0;
        }
        // Z_{a,i} = -(Z_aa A_{a,i} + Z_ab A_{b,i}) D_i^-1, Z_{b,i} = -(Z_ba A_{a,i} + Z_bb A_{b,i}) D_i^-1
        mm<HB>(zlt, Zaa, Ra + (size_t)i * BB);
        if (hb) mm_acc<HB>(zlt, 1.0, Zab, Rb + (size_t)i * BB);
        right_mul_inplace<HB>(zlt, Di);
        for (int e = 0; e < BB; ++e) zlt[e] = -zlt[e];
        if (hb) {
          mm<HB>(zrt, Zba, Ra + (size_t)i * BB);
          mm_acc<HB>(zrt, 1.0, Zbb, Rb + (size_t)i * BB);
          right_mul_inplace<HB>(zrt, Di);
          for (int e = 0; e < BB; ++e) zrt[e] = -zrt[e];
        } else {
          for (int e = 0; e < BB; ++e) zrt[e] = 0.0;
        }
        // Z_ii = D_i^-1 - X_a Z_{a,i} - X_b Z_{b,i}
        double* Zi = Zd + (size_t)i * BB;
        for (int e = 0; e < BB; ++e) Zi[e] = Di[e];
        mm_acc<HB>(Zi, -1.0, Xa, zlt);
        if (hb) mm_acc<HB>(Zi, -1.0, Xb, zrt);
      }
      __syncthreads();
    }
  }
  // ---- scalar band of the inverse
  for (int idx = threadIdx.x; idx < n * WD; idx += NT) {
    const int i = idx / WD, o = idx - i * WD - HB, j = i + o;
    double v = 0.0;
    if (j >= 0 && j < n) {
      const int bi = i / HB, bj = j / HB, r = i - bi * HB, c = j - bj * HB;
      if (bi == bj) {
        v = Zd[(size_t)bi * BB + r * HB + c];
      } else if (bj == bi + 1) {  // Z_{bi, bi+1}: held by whichever of the two is odd
        v = (bi & 1) ? ZR[(size_t)bi * BB + r * HB + c] : ZLt[(size_t)bj * BB + r * HB + c];
      } else {  // bj == bi - 1
        v = (bi & 1) ? ZL[(size_t)bi * BB + r * HB + c] : ZRt[(size_t)bj * BB + r * HB + c];
      }
    }
    zband[idx] = v;
  }
  __syncthreads();
  const bool ok = bad == 0;
  __syncthreads();
  return ok;
}

template <int NT>
__device__ double block_max(double v) {
  __shared__ double red[NT / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) t = fmax(t, red[i]);
  __syncthreads();
  return t;
}

// The matrix counts as numerically singular when its inverse's band holds an entry of
// 1e15 or more over the matrix's largest entry (a condition number whose error bound
// kappa u, u = 2^-53, reaches 0.1: no correct digit left in an FP64 inverse).
template <int NT>
__device__ bool band_well_conditioned(int count, const double* zband, double scale) {
  double m = 0.0;
  for (int i = threadIdx.x; i < count; i += NT) m = fmax(m, fabs(zband[i]));
  m = block_max<NT>(m);
  return m * scale < 1e15;
}

// Lattice coordinate of sample p of slice n (FP64, as in the gridding kernels).
template <typename R>
__device__ __forceinline__ double ffr_lam(const Geo& g, const Tab<R>& t, int n, int p) {
  return lattice_coord(kx_of(t, raw_k(t, g.n_freq, n, p), t.ku[n]), g);
}

// Full-rank route, one workgroup per slice (persistent over slices).  LDS: the W taps
// of every sample and its lattice floor.  The band of G~ goes to the workgroup's
// scratch, its selected inverse next to it, and B_r of that to D.
template <typename R, int HB, int NT>
__global__ __launch_bounds__(NT) void k_ffr_direct(Geo g, Tab<R> t, double* __restrict__ scratch, size_t per_wg,
                                                   R* __restrict__ dband, int* __restrict__ status) {
  constexpr int WD = 2 * HB + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  const int P = g.n_freq, K = (int)ceil(g.q) + 1, KT = 2 * K + 1, r = g.band_r;
  double* lw = reinterpret_cast<double*>(smem);  // [P][KT] W taps
  int* lfl = reinterpret_cast<int*>(lw + (size_t)P * KT);
  double* gb = scratch + per_wg * blockIdx.x;  // [P][WD] band of G~
  double* zb = gb + (size_t)P * WD;            // [P][WD] band of its inverse
  double* work = zb + (size_t)P * WD;
  for (int n = blockIdx.x; n < g.n_pulses; n += gridDim.x) {
    for (int p = threadIdx.x; p < P; p += NT) {
      double rp[kFfrMaxKT], rw[kFfrMaxKT];
      int fl;
      frame_taps(ffr_lam(g, t, n, p), g, K, rp, rw, fl);
      for (int k = 0; k < KT; ++k) lw[(size_t)p * KT + k] = rw[k];
      lfl[p] = fl;
    }
    __syncthreads();
    double scale = 0.0;
    for (int p = threadIdx.x; p < P; p += NT) {
      double rp[kFfrMaxKT], rw[kFfrMaxKT];
      int fl;
      frame_taps(ffr_lam(g, t, n, p), g, K, rp, rw, fl);
      for (int o = -HB; o <= HB; ++o) {
        const int pp = p + o;
        double acc = 0.0;
        if (pp >= 0 && pp < P) {
          const int sh = fl - lfl[pp];  // m = fl + k = fl[pp] + (k + sh)
          for (int k = 0; k < KT; ++k) {
            const int k2 = k + sh;
            if (k2 >= 0 && k2 < KT) acc += rp[k] * lw[(size_t)pp * KT + k2];
          }
        }
        gb[(size_t)p * WD + HB + o] = acc;
        scale = fmax(scale, fabs(acc));
      }
    }
    __syncthreads();
    scale = block_max<NT>(scale);
    bool ok = band_selinv<HB, NT>(P, gb, work, zb, 1e-13 * fmax(scale, 1e-300) + 1e-300);
    if (!ok && threadIdx.x == 0) atomicMax(status, 1);
    const bool wc = ok && band_well_conditioned<NT>(P * WD, zb, scale);
    if (ok && !wc && threadIdx.x == 0) atomicMax(status, 3);
    ok = ok && wc;
    R* D = dband + (size_t)n * P * (2 * r + 1);
    for (int idx = threadIdx.x; idx < P * (2 * r + 1); idx += NT) {
      const int p = idx / (2 * r + 1), o = idx - p * (2 * r + 1) - r;
      D[idx] = (ok && p + o >= 0 && p + o < P) ? (R)zb[(size_t)p * WD + HB + o] : (R)0;
    }
    __syncthreads();
  }
}

// Rank-deficient route (half-band 10 of Sa Sb for q <= 3), one workgroup per slice.
// Lattice points of slice n: l = l0 + j, j < L_n, with l0 = floor(lam_min - q) + 1 and
// every point within q of some sample.  Scratch per workgroup: the taps of every sample
// [P][2][KT] and floors, Sa and Sb bands [L][11], C = Sa Sb band [L][21], N band [L][21],
// the diagonal scaling [L], and the reduction's work.
constexpr int kFfrNHB = 10;  // half-band of Sa Sb (two half-bands 2q - 1 = 5)
template <typename R, int NT>
__global__ __launch_bounds__(NT) void k_ffr_normal(Geo g, Tab<R> t, double* __restrict__ scratch, size_t per_wg,
                                                   int lmax, R* __restrict__ dband, int* __restrict__ status) {
  constexpr int HB = kFfrNHB, WD = 2 * HB + 1, SH = 5, SW = 2 * SH + 1;
  const int P = g.n_freq, K = (int)ceil(g.q) + 1, KT = 2 * K + 1, r = g.band_r;
  __shared__ int l0_s, L_s;
  double* base = scratch + per_wg * blockIdx.x;
  double* tp = base;                              // [P][KT] R_Psi taps
  double* tw = tp + (size_t)P * KT;               // [P][KT] R_W taps
  int* fl = reinterpret_cast<int*>(tw + (size_t)P * KT);  // [P] lattice floors
  double* sa = tw + (size_t)P * KT + (P + 1) / 2;  // [lmax][SW]
  double* sb = sa + (size_t)lmax * SW;             // [lmax][SW]
  double* cb = sb + (size_t)lmax * SW;             // [lmax][WD]
  double* nb_ = cb + (size_t)lmax * WD;            // [lmax][WD]
  double* sc = nb_ + (size_t)lmax * WD;            // [lmax] 1 / s_j
  double* work = sc + lmax;
  for (int n = blockIdx.x; n < g.n_pulses; n += gridDim.x) {
    for (int p = threadIdx.x; p < P; p += NT) {
      double rp[kFfrMaxKT], rw[kFfrMaxKT];
      int f;
      frame_taps(ffr_lam(g, t, n, p), g, K, rp, rw, f);
      for (int k = 0; k < KT; ++k) {
        tp[(size_t)p * KT + k] = rp[k];
        tw[(size_t)p * KT + k] = rw[k];
      }
      fl[p] = f;
    }
    if (threadIdx.x == 0) {
      const double lmin = ffr_lam(g, t, n, 0), lmx = ffr_lam(g, t, n, P - 1);
      l0_s = (int)floor(lmin - g.q) + 1;
      L_s = (int)(ceil(lmx + g.q) - 1.0) - l0_s + 1;
    }
    __syncthreads();
    const int l0 = l0_s, L = L_s;
    if (L > lmax || L < 1) {  // cannot happen with the plan's margin; refuse rather than overrun
      if (threadIdx.x == 0) atomicMax(status, 2);
      __syncthreads();
      continue;
    }
    // Gram bands: Sa[l][l + o] = sum_p A[p][l] A[p][l + o] (o in [-5, 5]), Sb likewise.
    // Point l is reached by the samples whose floors lie in [l - K, l + K]: found by
    // binary search (floors rise along the slice).
    for (int j = threadIdx.x; j < L; j += NT) {
      const int l = l0 + j;
      int lo = 0, hi = P;  // first p with fl[p] >= l - K
      while (lo < hi) {
        const int mid = (lo + hi) / 2;
        if (fl[mid] < l - K) lo = mid + 1; else hi = mid;
      }
      double accA[SW], accB[SW];
      for (int o = 0; o < SW; ++o) accA[o] = accB[o] = 0.0;
      for (int p = lo; p < P && fl[p] <= l + K; ++p) {
        const int k = l - fl[p] + K;  // tap index of l for sample p
        const double ap = tp[(size_t)p * KT + k], bp = tw[(size_t)p * KT + k];
        if (ap == 0.0 && bp == 0.0) continue;
        for (int o = -SH; o <= SH; ++o) {
          const int k2 = k + o;
          if (k2 >= 0 && k2 < KT) {
            accA[o + SH] += ap * tp[(size_t)p * KT + k2];
            accB[o + SH] += bp * tw[(size_t)p * KT + k2];
          }
        }
      }
      for (int o = 0; o < SW; ++o) {
        const bool in = j + o - SH >= 0 && j + o - SH < L;
        sa[(size_t)j * SW + o] = in ? accA[o] : 0.0;
        sb[(size_t)j * SW + o] = in ? accB[o] : 0.0;
      }
    }
    __syncthreads();
    // C = Sa Sb, half-band 10, and its diagonal scaling s_j = sqrt|C_jj|
    for (int j = threadIdx.x; j < L; j += NT) {
      for (int o = -HB; o <= HB; ++o) {
        const int jj = j + o;
        double acc = 0.0;
        if (jj >= 0 && jj < L)
          for (int m = max(j - SH, jj - SH); m <= min(j + SH, jj + SH); ++m)
            if (m >= 0 && m < L) acc += sa[(size_t)j * SW + (m - j + SH)] * sb[(size_t)m * SW + (jj - m + SH)];
        cb[(size_t)j * WD + HB + o] = acc;
      }
      const double dj = sqrt(fabs(cb[(size_t)j * WD + HB]));
      sc[j] = dj > 0.0 ? 1.0 / dj : 1.0;
    }
    __syncthreads();
    // Equilibrate: C^ = S^-1 C S^-1.  Lattice points near the slice ends are reached by few
    // samples with small taps, so C's rows differ in scale by up to ~1e7; the reduction and
    // its pivot and conditioning checks then see the intrinsic conditioning of the
    // product (N = S^-1 (C^)^-1 S^-1 below).
    double scale = 0.0;
    for (int idx = threadIdx.x; idx < L * WD; idx += NT) {
      const int j = idx / WD, jj = j + idx - j * WD - HB;
      if (jj >= 0 && jj < L) {
        cb[idx] *= sc[j] * sc[jj];
        scale = fmax(scale, fabs(cb[idx]));
      }
    }
    __syncthreads();
    scale = block_max<NT>(scale);
    bool ok = band_selinv<HB, NT>(L, cb, work, nb_, 1e-13 * fmax(scale, 1e-300) + 1e-300);
    if (!ok && threadIdx.x == 0) atomicMax(status, 1);
    const bool wc = ok && band_well_conditioned<NT>(L * WD, nb_, scale);
    if (ok && !wc && threadIdx.x == 0) atomicMax(status, 3);
    ok = ok && wc;
    // D[p][p + o] = sum_{l, l'} R_W(l - lam_p) N[l][l'] R_Psi(l' - lam_{p+o})
    R* D = dband + (size_t)n * P * (2 * r + 1);
    for (int idx = threadIdx.x; idx < P * (2 * r + 1); idx += NT) {
      const int p = idx / (2 * r + 1), o = idx - p * (2 * r + 1) - r, pp = p + o;
      double acc = 0.0;
      if (ok && pp >= 0 && pp < P) {
        for (int k = 0; k < KT; ++k) {
          const double bw = tw[(size_t)p * KT + k];
          if (bw == 0.0) continue;
          const int j = fl[p] - K + k - l0;
          for (int k2 = 0; k2 < KT; ++k2) {
            const double ap = tp[(size_t)pp * KT + k2];
            if (ap == 0.0) continue;
            const int jj = fl[pp] - K + k2 - l0;
            if (jj - j >= -HB && jj - j <= HB) acc += bw * (sc[j] * nb_[(size_t)j * WD + HB + (jj - j)] * sc[jj]) * ap;
          }
        }
      }
      D[idx] = (R)acc;
    }
    __syncthreads();
  }
}

// ============================================================================ launchers
#ifdef TFFR_EMIT_SHARED
size_t ffr_scratch_bytes(const Geo& g, int route, int lmax, int nwg) {
  const int K = (int)ceil(g.q) + 1, KT = 2 * K + 1, P = g.n_freq;
  size_t per;
  if (route == 0) {
    const int HB = g.band_b, nb = (P + HB - 1) / HB;
    per = 2 * (size_t)P * (2 * HB + 1) + 10 * (size_t)nb * HB * HB;
  } else {
    const int HB = kFfrNHB, nb = (lmax + HB - 1) / HB;
    per = 2 * (size_t)P * KT + (P + 1) / 2 + 2 * (size_t)lmax * 11 + 2 * (size_t)lmax * (2 * HB + 1) + lmax +
          10 * (size_t)nb * HB * HB;
  }
  return per * nwg * sizeof(double);
}
#endif

template <typename R>
hipError_t launch_ffr(const Geo& g, const Tab<R>& t, int route, int lmax, int nwg, double* scratch, R* dband,
                      int* status, hipStream_t st) {
  constexpr int NT = 256;
  const size_t per = ffr_scratch_bytes(g, route, lmax, 1) / sizeof(double);
  if (route == 1) {
    auto fn = k_ffr_normal<R, NT>;
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(NT), 0, st, g, t, scratch, per, lmax, dband, status);
    return hipGetLastError();
  }
  const int K = (int)ceil(g.q) + 1, KT = 2 * K + 1;
  const size_t lds = (size_t)g.n_freq * (KT * sizeof(double) + sizeof(int));
#define TFFR_FFR_DIRECT(BB)                                                                   \
  case BB: {                                                                                  \
    auto fn = k_ffr_direct<R, BB, NT>;                                                        \
    hipError_t e = allow_lds((const void*)fn, lds);                                           \
    if (e != hipSuccess) return e;                                                            \
    hipLaunchKernelGGL(fn, dim3(nwg), dim3(NT), lds, st, g, t, scratch, per, dband, status);  \
    return hipGetLastError();                                                                 \
  }
  switch (g.band_b) {
    TFFR_FFR_DIRECT(1)
    TFFR_FFR_DIRECT(2)
    TFFR_FFR_DIRECT(3)
    TFFR_FFR_DIRECT(4)
    TFFR_FFR_DIRECT(5)
    TFFR_FFR_DIRECT(6)
    TFFR_FFR_DIRECT(7)
    TFFR_FFR_DIRECT(8)
    default:
      return hipErrorInvalidValue;
  }
#undef TFFR_FFR_DIRECT
}

#define TFFR_INSTANTIATE(R) \
  template hipError_t launch_ffr<R>(const Geo&, const Tab<R>&, int, int, int, double*, R*, int*, hipStream_t);

TFFR_INSTANTIATE_TYPES

}  // namespace tffr
