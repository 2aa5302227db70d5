// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64) with LDS-staged 64x64x16 tiles, and the
// column-dot reduction used for Phi(X)_i = R[:,i]^T (X R)[:,i] and the diagonal extract of the CG matvec.
#include "kot_internal.h"
#include <algorithm>
#include <map>
#include <mutex>
#include <tuple>

namespace kot {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int KM_S = BM + 2;   // k-major tile [BK][KM_S] (operand loaded along m / n)
constexpr int MK_S = BK + 1;   // m-major tile [BM][MK_S] (operand loaded along k)
constexpr int TILE_D = BK * KM_S;  // == BM * MK_S == 2112 doubles either way
static_assert(BK * KM_S == BM * MK_S, "tile sizes");

// One 64x64 output tile per workgroup.  The workgroup has NW = (4/FM)(4/FN) waves; each wave owns a
// (16 FM) x (16 FN) block of FM x FN MFMA tiles of 16x16 (FM = FN = 2: 4 waves of 32x32; FM = 1, FN = 2:
// 8 waves; FM = FN = 1: 16 waves).  More waves per SIMD keep the FP64 matrix pipeline fed when the grid
// has about one tile per CU.  MFMA operand layout (16x16x4 f64): lane L supplies A[L%16][L/16] and
// B[L/16][L%16]; the accumulator lane L holds D[L/16 + 4*v][L%16], v = 0..3.
// Each operand is staged in LDS along the dimension it is contiguous in (global loads and LDS stores both
// run along that dimension; the odd row stride of the m-major layout keeps the 16-row MFMA reads
// conflict-free).  The next 32-deep K slice is prefetched into registers while the current one feeds the
// matrix cores.
template <bool TA, bool TB, bool SC, int NT>
struct Tile {
  static constexpr int PER = BM * BK / NT;     // elements of each operand per thread and K slice
  static constexpr int RK = NT / BK;           // rows per pass when lanes run along k
  static constexpr int RM = NT / BM;           // k-rows per pass when lanes run along m / n
  double a[PER], b[PER];
  __device__ __forceinline__ void load(const GemmArgs& g, const double* __restrict__ A, const double* __restrict__ B,
                                       const double* __restrict__ S, int m0, int n0, int k0, int t) {
    const int M = g.m, N = g.n, K = g.k;
    if (!TA) {  // A[m*lda + k]: lanes along k (32)
      const int kk = t & (BK - 1), mm = t / BK;
      const int gk = k0 + kk;
      const double sc = (SC && gk < K) ? S[gk] : 1.0;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int gm = m0 + mm + RK * u;
        const double v = (gm < M && gk < K) ? A[(long long)gm * g.lda + gk] : 0.0;
        a[u] = SC ? v * sc : v;
      }
    } else {    // A[k*lda + m]: lanes along m (64)
      const int mm = t & (BM - 1), kk = t / BM;
      const int gm = m0 + mm;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int gk = k0 + kk + RM * u;
        const double v = (gm < M && gk < K) ? A[(long long)gk * g.lda + gm] : 0.0;
        a[u] = SC ? ((gk < K) ? v * S[gk] : 0.0) : v;
      }
    }
    if (!TB) {  // B[k*ldb + n]: lanes along n
      const int nn = t & (BN - 1), kk = t / BN;
      const int gn = n0 + nn;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int gk = k0 + kk + RM * u;
        b[u] = (gn < N && gk < K) ? B[(long long)gk * g.ldb + gn] : 0.0;
      }
    } else {    // B[n*ldb + k]: lanes along k
      const int kk = t & (BK - 1), nn = t / BK;
      const int gk = k0 + kk;
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int gn = n0 + nn + RK * u;
        b[u] = (gn < N && gk < K) ? B[(long long)gn * g.ldb + gk] : 0.0;
      }
    }
  }
  __device__ __forceinline__ void store(double* __restrict__ As, double* __restrict__ Bs, int t) const {
    if (!TA) {  // m-major
      const int kk = t & (BK - 1), mm = t / BK;
#pragma unroll
      for (int u = 0; u < PER; ++u) As[(mm + RK * u) * MK_S + kk] = a[u];
    } else {    // k-major
      const int mm = t & (BM - 1), kk = t / BM;
#pragma unroll
      for (int u = 0; u < PER; ++u) As[(kk + RM * u) * KM_S + mm] = a[u];
    }
    if (!TB) {  // k-major
      const int nn = t & (BN - 1), kk = t / BN;
#pragma unroll
      for (int u = 0; u < PER; ++u) Bs[(kk + RM * u) * KM_S + nn] = b[u];
    } else {    // n-major
      const int kk = t & (BK - 1), nn = t / BK;
#pragma unroll
      for (int u = 0; u < PER; ++u) Bs[(nn + RK * u) * MK_S + kk] = b[u];
    }
  }
  // op(A)[m][k] and op(B)[k][n] from the staged tiles
  static __device__ __forceinline__ double ga(const double* As, int m, int k) {
    return TA ? As[k * KM_S + m] : As[m * MK_S + k];
  }
  static __device__ __forceinline__ double gb(const double* Bs, int k, int n) {
    return TB ? Bs[n * MK_S + k] : Bs[k * KM_S + n];
  }
};

// K range [klo, khi) of output tile (m0, n0) where the triangular operands (bits of tri) can be nonzero,
// klo aligned down to BK.
__device__ __forceinline__ void tri_k_range(int tri, int k, int m0, int n0, int& klo, int& khi) {
  klo = 0;
  khi = k;
  if (tri & 1) klo = max(klo, m0);            // op(A) upper: op(A)[m][k] = 0 for k < m
  if (tri & 8) klo = max(klo, n0);            // op(B) lower: op(B)[k][n] = 0 for k < n
  if (tri & 2) khi = min(khi, m0 + BM);       // op(A) lower: zero for k > m
  if (tri & 4) khi = min(khi, n0 + BN);       // op(B) upper: zero for k > n
  klo &= ~(BK - 1);
}

// blockIdx.z = batch * splits + split.  With splits > 1 the workgroup covers K slices
// [split*kchunk, (split+1)*kchunk) and writes its raw partial tile to part (layout [batch][split][m][n]); a
// split that misses the tile's K range writes nothing (the reduction skips it the same way).
// With a work list (units != null, a 1D grid) workgroup i takes entry i: (tile row << 16) | (tile col << 8) | K
// slice, or -1 for nothing.
template <bool TA, bool TB, bool SC, int FM, int FN>
__global__ __launch_bounds__(64 * (4 / FM) * (4 / FN)) void gemm_f64_kernel(GemmArgs g, int splits, int kchunk,
                                                                             double* __restrict__ part,
                                                                             const int* __restrict__ units) {
  constexpr int WN = 4 / FN;                   // waves along n
  constexpr int NT = 64 * (4 / FM) * WN;
  __shared__ double As2[2][TILE_D];  // two K slices in LDS: one feeds the matrix cores while the next is stored
  __shared__ double Bs2[2][TILE_D];
  int bz, sp, m0, n0;
  if (units) {
    const int u = units[blockIdx.x];
    if (u < 0) return;
    bz = 0;
    sp = u & 255;
    m0 = (u >> 16) * BM;
    n0 = ((u >> 8) & 255) * BN;
  } else {
    bz = blockIdx.z / splits;
    sp = blockIdx.z % splits;
    m0 = blockIdx.y * BM;
    n0 = blockIdx.x * BN;
  }
  const double* __restrict__ A = g.A + bz * g.sA;
  const double* __restrict__ B = g.B + bz * g.sB;
  const double* __restrict__ S = SC ? g.s + bz * g.sS : nullptr;
  double* __restrict__ C = g.C + bz * g.sC;
  if (g.lower && n0 > m0 + BM - 1) return;  // tile strictly above the diagonal (uniform per workgroup)
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave / WN, wn = wave % WN;
  // K range of this split, narrowed to where the triangular operands can be nonzero for this tile
  int klo, khi;
  tri_k_range(g.tri, g.k, m0, n0, klo, khi);
  const int kbeg = max(sp * kchunk, klo);
  const int kend = min(min(g.k, sp * kchunk + kchunk), khi);
  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (splits > 1 && nk == 0) return;  // nothing of this tile in this split (uniform per workgroup)
  using T = Tile<TA, TB, SC, NT>;

  dbl4 acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  // Two register sets of loads in flight: slice kt + 2 is requested while slice kt feeds the matrix cores and
  // slice kt + 1 (requested one slice earlier) goes to the other LDS buffer, so each global load has two
  // slices of compute to arrive.
  T tile0, tile1;
  GemmArgs gk = g;
  gk.k = kend;  // bounds for the loads of this split
  tile0.load(gk, A, B, S, m0, n0, kbeg, t);
  tile0.store(As2[0], Bs2[0], t);
  if (nk > 1) tile1.load(gk, A, B, S, m0, n0, kbeg + BK, t);
  __syncthreads();
  const int r16 = lane & 15, k4 = lane >> 4;
  // spare: its slice kt is in LDS already, so it takes the request for slice kt + 2; next holds slice kt + 1
  auto step = [&](int kt, T& spare, T& next) {
    const double* As = As2[kt & 1];
    const double* Bs = Bs2[kt & 1];
    if (kt + 2 < nk) spare.load(gk, A, B, S, m0, n0, kbeg + (kt + 2) * BK, t);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = T::ga(As, wm * 16 * FM + i * 16 + r16, ks + k4);
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = T::gb(Bs, ks + k4, wn * 16 * FN + j * 16 + r16);
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    // slice kt + 1 goes to the other buffer; one barrier then both publishes it and ends every read of this
    // one, which slice kt + 2 overwrites
    if (kt + 1 < nk) {
      next.store(As2[(kt + 1) & 1], Bs2[(kt + 1) & 1], t);
      __syncthreads();
    }
  };
  for (int kt = 0; kt < nk; kt += 2) {  // two slices per pass, so that each register set stays in place
    step(kt, tile0, tile1);
    if (kt + 1 < nk) step(kt + 1, tile1, tile0);
  }
  // ---- epilogue ----
  const int M = g.m, N = g.n;
  if (g.D) {
    // column-dot mode: sum_i D_ij (alpha acc)_ij over this tile's rows, per column, into part[(tile row, split)]:
    // over each lane's rows, then the four lanes of a column (k4), then the row-group waves in order
    __shared__ double dsum[4 / FM][BN];
    double cs[FN];
#pragma unroll
    for (int j = 0; j < FN; ++j) {
      cs[j] = 0.0;
      const int col = n0 + wn * 16 * FN + j * 16 + r16;
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = m0 + wm * 16 * FM + i * 16 + k4 + 4 * v;
          if (row < M && col < N) cs[j] += g.D[(long long)row * g.ldd + col] * (g.alpha * acc[i][j][v]);
        }
      cs[j] += __shfl_xor(cs[j], 16);
      cs[j] += __shfl_xor(cs[j], 32);
      if (k4 == 0) dsum[wm][wn * 16 * FN + j * 16 + r16] = cs[j];
    }
    __syncthreads();
    if ((int)threadIdx.x < BN && n0 + (int)threadIdx.x < N) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < 4 / FM; ++w) s += dsum[w][threadIdx.x];
      part[((long long)(m0 / BM) * splits + sp) * N + n0 + threadIdx.x] = s;
    }
    return;
  }
  // strictly lower tile of a symmetric result: the transpose goes out through LDS, row segments again
  const bool mir = splits == 1 && g.mirror && n0 < m0;
  double* Tt = &As2[0][0];  // 64 x 65 staging tile (the K loop's buffers are free once every wave is past it)
  if (mir) __syncthreads();
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 16 * FM + i * 16 + k4 + 4 * v;
        const int col = n0 + wn * 16 * FN + j * 16 + r16;
        if (row < M && col < N) {
          if (splits > 1) {
            part[(((long long)bz * splits + sp) * M + row) * N + col] = acc[i][j][v];
          } else {
            double* p = C + (long long)row * g.ldc + col;
            const double r = g.alpha * acc[i][j][v];
            *p = (g.beta == 0.0) ? r : r + g.beta * (*p);
            if (mir) Tt[(row - m0) * (BN + 1) + (col - n0)] = r;
          }
        }
      }
  if (mir) {
    __syncthreads();
    for (int e = (int)threadIdx.x; e < BM * BN; e += NT) {
      const int a = e / BM, b = e % BM;  // C[n0 + a][m0 + b] = tile[b][a]
      if (n0 + a < N && m0 + b < M) {
        double* q = C + (long long)(n0 + a) * g.ldc + (m0 + b);
        const double r = Tt[b * (BN + 1) + a];
        *q = (g.beta == 0.0) ? r : r + g.beta * (*q);
      }
    }
  }
}

// C = alpha * sum_s part[b][s] + beta * C, summed in split order over the splits that met the tile's K range;
// one 16-row slab of a 64 x 64 tile per workgroup (row segments in and out; many workgroups keep enough loads
// in flight), the transpose of a slab of a strictly lower tile of a symmetric result written through LDS as
// 128-byte row segments too.
constexpr int RS = 16;  // rows per reduction slab
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g, int splits, int kchunk,
                                                            const double* __restrict__ part) {
  __shared__ double Tt[RS][BN + 1];
  const int s0 = blockIdx.y * RS, n0 = blockIdx.x * BN, bz = blockIdx.z;
  const int m0 = (s0 / BM) * BM;  // the slab's GEMM tile row
  if (g.lower && n0 > m0 + BM - 1) return;  // tile above the diagonal: not computed (uniform per workgroup)
  int klo, khi;
  tri_k_range(g.tri, g.k, m0, n0, klo, khi);
  const long long mn = (long long)g.m * g.n;
  const double* pb = part + (long long)bz * splits * mn;
  double* Cb = g.C + bz * g.sC;
  const int t = threadIdx.x, cc = t & (BN - 1);
  const bool mir = g.mirror && n0 < m0;
  const int col = n0 + cc, colc = min(col, g.n - 1);
  constexpr int E = RS / 4;  // elements per thread
  double s[E];
#pragma unroll
  for (int q = 0; q < E; ++q) s[q] = 0.0;
  for (int sp = 0; sp < splits; ++sp) {
    if (!(max(sp * kchunk, klo) < min(min(g.k, sp * kchunk + kchunk), khi))) continue;  // uniform
    const double* ps = pb + sp * mn;
    double v[E];
#pragma unroll
    for (int q = 0; q < E; ++q) v[q] = ps[(long long)min(s0 + (t >> 6) + 4 * q, g.m - 1) * g.n + colc];
#pragma unroll
    for (int q = 0; q < E; ++q) s[q] += v[q];
  }
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int rr = (t >> 6) + 4 * q;
    const int row = s0 + rr;
    if (row < g.m && col < g.n) {
      double* c = Cb + (long long)row * g.ldc + col;
      const double r = g.alpha * s[q];
      *c = (g.beta == 0.0) ? r : r + g.beta * (*c);
      if (mir) Tt[rr][cc] = r;
    }
  }
  if (!mir) return;
  __syncthreads();
#pragma unroll
  for (int q = 0; q < E; ++q) {
    const int a = (t >> 4) + 16 * q, b = t & (RS - 1);  // C[n0 + a][s0 + b] = slab[b][a]
    if (n0 + a < g.n && s0 + b < g.m) {
      double* d = Cb + (long long)(n0 + a) * g.ldc + (s0 + b);
      const double r = Tt[b][a];
      *d = (g.beta == 0.0) ? r : r + g.beta * (*d);
    }
  }
}

// Column-dot mode's sum: y_j = dalpha sum over tile rows and the splits that met each tile's K range of part +
// dbeta y_j.  64 columns per workgroup; the (tile row, split) terms of a column are dealt round-robin to four
// thread groups and the four group sums added in order (a fixed order throughout).
__global__ __launch_bounds__(256) void coldot_final_kernel(GemmArgs g, int splits, int kchunk,
                                                           const double* __restrict__ part) {
  __shared__ double gs[4][64];
  const int t = threadIdx.x, c = t & 63, grp = t >> 6;
  const int col = blockIdx.x * 64 + c;
  const int n0 = blockIdx.x * 64, mt = (g.m + BM - 1) / BM;
  const int colc = min(col, g.n - 1);
  double s = 0.0;
  for (int q = grp; q < mt * splits; q += 4) {
    const int tr = q / splits, sp = q - tr * splits;
    int klo, khi;
    tri_k_range(g.tri, g.k, tr * BM, n0, klo, khi);
    if (max(sp * kchunk, klo) < min(min(g.k, sp * kchunk + kchunk), khi)) s += part[(long long)q * g.n + colc];
  }
  gs[grp][c] = s;
  __syncthreads();
  if (grp == 0 && col < g.n) {
    const double v = (gs[0][c] + gs[1][c]) + (gs[2][c] + gs[3][c]);
    g.y[col] = (g.dbeta == 0.0) ? g.dalpha * v : g.dalpha * v + g.dbeta * g.y[col];
  }
}

// y[r] = alpha * sum_k A[r][k] s[k] x[k] + beta * y[r]: one wavefront per row (loads along k), fixed-order
// lane partials and a butterfly reduction, so the result does not depend on the launch.
__global__ __launch_bounds__(256) void gemv_f64_kernel(int m, int k, double alpha, const double* __restrict__ A, int lda,
                                                        const double* __restrict__ s, const double* __restrict__ x, int incx,
                                                        double beta, double* __restrict__ y, int incy) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;  // uniform per wavefront
  const double* __restrict__ a = A + (long long)row * lda;
  // four independent lane partials (four loads of the row in flight), combined in a fixed order
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  int c = lane;
  for (; c + 192 < k; c += 256) {
    double av[4], xv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = a[c + 64 * u];
      const long long cx = (long long)(c + 64 * u);
      xv[u] = s ? s[cx] * x[cx * incx] : x[cx * incx];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] += av[u] * xv[u];
  }
  for (; c < k; c += 64) q[0] += a[c] * (s ? s[c] * x[(long long)c * incx] : x[(long long)c * incx]);
  double acc = (q[0] + q[1]) + (q[2] + q[3]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    double* p = y + (long long)row * incy;
    *p = (beta == 0.0) ? alpha * acc : alpha * acc + beta * (*p);
  }
}

// Row-vector products (m = 1): c_j = sum_k a_k s_k op(B)_kj with a_k = op(A)_0k.  The epilogue writes
// C_0j = alpha c_j + beta C_0j, or in column-dot mode y_j = dalpha D_0j (alpha c_j) + dbeta y_j.
__device__ __forceinline__ void rowvec_store(int j, double v, double alpha, double beta, double* __restrict__ C,
                                             const double* __restrict__ D, double dalpha, double dbeta,
                                             double* __restrict__ y) {
  if (D) {
    const double w = D[j] * (alpha * v);
    y[j] = (dbeta == 0.0) ? dalpha * w : dalpha * w + dbeta * y[j];
  } else {
    C[j] = (beta == 0.0) ? alpha * v : alpha * v + beta * C[j];
  }
}

// op(B)_kj = B[j * ldb + k] (k <= kRowvecMaxK): the workgroup stages x_k = s_k a_k in LDS once, then one
// wavefront per output j reads its row of B along k with eight loads in flight per lane; the lane partials are
// combined in a fixed order, then a butterfly.
constexpr int kRowvecMaxK = 4096;
__global__ __launch_bounds__(256) void rowvec_dot_kernel(int n, int k, const double* __restrict__ a, int inca,
                                                         const double* __restrict__ s, const double* __restrict__ B,
                                                         int ldb, double alpha, double beta, double* __restrict__ C,
                                                         const double* __restrict__ D, double dalpha, double dbeta,
                                                         double* __restrict__ y) {
  __shared__ double xs[kRowvecMaxK];
  for (int kk = threadIdx.x; kk < k; kk += 256)
    xs[kk] = s ? s[kk] * a[(long long)kk * inca] : a[(long long)kk * inca];
  __syncthreads();
  const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= n) return;  // uniform per wavefront (after the barrier)
  const double* __restrict__ b = B + (long long)j * ldb;
  double q[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int kk = lane;
  for (; kk + 448 < k; kk += 512) {
    double bv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) bv[u] = b[kk + 64 * u];
#pragma unroll
    for (int u = 0; u < 8; ++u) q[u] += xs[kk + 64 * u] * bv[u];
  }
  for (; kk < k; kk += 64) q[0] += xs[kk] * b[kk];
  double acc = ((q[0] + q[1]) + (q[2] + q[3])) + ((q[4] + q[5]) + (q[6] + q[7]));
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) rowvec_store(j, acc, alpha, beta, C, D, dalpha, dbeta, y);
}

// op(B)_kj = B[k * ldb + j]: workgroup (x, z) sums K slice z of 64 columns, the four thread groups taking every
// fourth k of the slice (four loads in flight each), and writes part[z][j].
__global__ __launch_bounds__(256) void rowvec_colsum_kernel(int n, int k, int kc, const double* __restrict__ a,
                                                            int inca, const double* __restrict__ s,
                                                            const double* __restrict__ B, int ldb,
                                                            double* __restrict__ part) {
  __shared__ double red[4][64];
  const int t = threadIdx.x, c = t & 63, grp = t >> 6;
  const int j = blockIdx.x * 64 + c;
  const int k0 = blockIdx.y * kc, k1 = min(k, k0 + kc);
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  if (j < n) {
    int kk = k0 + grp;
    for (; kk + 12 < k1; kk += 16) {
      double bv[4], xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int kq = kk + 4 * u;
        bv[u] = B[(long long)kq * ldb + j];
        xv[u] = s ? s[kq] * a[(long long)kq * inca] : a[(long long)kq * inca];
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) q[u] += xv[u] * bv[u];
    }
    for (; kk < k1; kk += 4) q[0] += (s ? s[kk] * a[(long long)kk * inca] : a[(long long)kk * inca]) * B[(long long)kk * ldb + j];
  }
  red[grp][c] = (q[0] + q[1]) + (q[2] + q[3]);
  __syncthreads();
  if (grp == 0 && j < n) part[(long long)blockIdx.y * n + j] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
}

// Sums the K slices of rowvec_colsum_kernel in slice order (ks <= kRowvecMaxSlices, every load issued before
// the sum) and applies the epilogue.
constexpr int kRowvecMaxSlices = 64;
__global__ __launch_bounds__(256) void rowvec_final_kernel(int n, int ks, const double* __restrict__ part, double alpha,
                                                           double beta, double* __restrict__ C,
                                                           const double* __restrict__ D, double dalpha, double dbeta,
                                                           double* __restrict__ y) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  double pv[kRowvecMaxSlices];
#pragma unroll
  for (int z = 0; z < kRowvecMaxSlices; ++z) pv[z] = z < ks ? part[(long long)z * n + j] : 0.0;
  double v = 0.0;
#pragma unroll
  for (int z = 0; z < kRowvecMaxSlices; ++z) v += pv[z];
  rowvec_store(j, v, alpha, beta, C, D, dalpha, dbeta, y);
}

// Rank-one products (k = 1): C_ij = alpha op(A)_i0 s_0 op(B)_0j + beta C_ij over the whole matrix, or over its
// lower triangle (lower), or over the lower triangle with each value also written to its mirror (lower and
// mirror; beta = 0 there, so no element is read after another thread wrote it).
__global__ __launch_bounds__(256) void rank1_kernel(int m, int n, double alpha, const double* __restrict__ A, int inca,
                                                    const double* __restrict__ s, const double* __restrict__ B, int incb,
                                                    double beta, double* __restrict__ C, int ldc, int lower,
                                                    int mirror) {
  const int j = blockIdx.x * 64 + (threadIdx.x & 63);
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= m || j >= n) return;
  const double s0 = s ? s[0] : 1.0;
  if (lower && j > i) {
    if (!mirror) return;
    // the mirror of (j, i), which lies in the lower triangle (j < m since j > i and the product is square)
    C[(long long)i * ldc + j] = alpha * ((A[(long long)j * inca] * s0) * B[(long long)i * incb]);
    return;
  }
  const double v = alpha * ((A[(long long)i * inca] * s0) * B[(long long)j * incb]);
  double* p = C + (long long)i * ldc + j;
  *p = (beta == 0.0) ? v : v + beta * (*p);
}

// y_r = a (Q v)_r + b (K2 v)_r + c v_r (K2 may be null): the Schur operator's dense part in one pass, one
// wavefront per row, four partial sums per lane for each product, combined in a fixed order.
__global__ __launch_bounds__(256) void gemv2_f64_kernel(int m, const double* __restrict__ Q, double a,
                                                         const double* __restrict__ K2, double b,
                                                         const double* __restrict__ v, double c,
                                                         double* __restrict__ y) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= m) return;  // uniform per wavefront
  const double* __restrict__ q = Q + (long long)row * m;
  const double* __restrict__ k2 = K2 ? K2 + (long long)row * m : nullptr;
  double p[4] = {0.0, 0.0, 0.0, 0.0}, r[4] = {0.0, 0.0, 0.0, 0.0};
  int j = lane;
  for (; j + 192 < m; j += 256) {
    double qv[4], kv[4], vv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      qv[u] = q[j + 64 * u];
      kv[u] = k2 ? k2[j + 64 * u] : 0.0;
      vv[u] = v[j + 64 * u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      p[u] += qv[u] * vv[u];
      r[u] += kv[u] * vv[u];
    }
  }
  for (; j < m; j += 64) {
    p[0] += q[j] * v[j];
    if (k2) r[0] += k2[j] * v[j];
  }
  double sq = (p[0] + p[1]) + (p[2] + p[3]);
  double sk = (r[0] + r[1]) + (r[2] + r[3]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sq += __shfl_xor(sq, off);
    sk += __shfl_xor(sk, off);
  }
  if (lane == 0) y[row] = a * sq + (K2 ? b * sk : 0.0) + c * v[row];
}

// Column dots: partial sums over kDiagParts row slabs, then a fixed-order sum -> deterministic.
__global__ __launch_bounds__(256) void diag_dot_part(int r0, int r1, int n, const double* __restrict__ A, int lda,
                                                      const double* __restrict__ B, int ldb, double* __restrict__ part) {
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int sub = threadIdx.x >> 6;  // 4 row interleaves inside the slab
  const int slab = blockIdx.y;
  const int rows = r1 - r0;
  const int per = (rows + kDiagParts - 1) / kDiagParts;
  const int s0 = r0 + slab * per;
  const int s1 = min(r1, s0 + per);
  double acc = 0.0;
  if (col < n)
    for (int r = s0 + sub; r < s1; r += 4) acc += A[(long long)r * lda + col] * B[(long long)r * ldb + col];
  __shared__ double red[4][64];
  red[sub][threadIdx.x & 63] = acc;
  __syncthreads();
  if (sub == 0 && col < n)
    part[(long long)slab * n + col] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}

__global__ void diag_dot_final(int n, double alpha, double beta, const double* __restrict__ part, double* __restrict__ y) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n) return;
  double s = 0.0;
#pragma unroll
  for (int p = 0; p < kDiagParts; ++p) s += part[(long long)p * n + col];
  y[col] = (beta == 0.0) ? alpha * s : alpha * s + beta * y[col];
}

}  // namespace

thread_local Profiler* g_prof = nullptr;
thread_local double* g_gemm_ws = nullptr;
thread_local size_t g_gemm_ws_cap = 0;
thread_local const int* g_gemm_tune = nullptr;

hipEvent_t Profiler::get() {
  if (next == pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[next++];
}
thread_local int g_prof_chain = 0;
void Profiler::begin(hipStream_t st, int cls, double flops, double bytes) {
  if (g_prof_chain && cls == PROF_GEMM_F64) cls = PROF_CHAIN_F64;
  Rec r{cls, flops, bytes, get(), get()};
  if (r.a) hipEventRecord(r.a, st);
  recs.push_back(r);
}
void Profiler::end(hipStream_t st) {
  if (!recs.empty() && recs.back().b) hipEventRecord(recs.back().b, st);
}
void Profiler::clear() { recs.clear(); next = 0; }
Profiler::~Profiler() { for (auto e : pool) hipEventDestroy(e); }

// Multiply-add work of one call as the kernel schedules it: 2 x rows x cols x (K range) summed over the
// output tiles it computes (tiles skipped by `lower` and K ranges cut by `tri` excluded).
static double gemm_work_flops(const GemmArgs& g) {
  if (!g.lower && !g.tri) return 2.0 * g.m * g.n * (double)g.k * g.batch;
  double fl = 0.0;
  for (int m0 = 0; m0 < g.m; m0 += BM)
    for (int n0 = 0; n0 < g.n; n0 += BN) {
      if (g.lower && n0 > m0 + BM - 1) continue;
      int klo = 0, khi = g.k;
      if (g.tri & 1) klo = std::max(klo, m0);
      if (g.tri & 8) klo = std::max(klo, n0);
      if (g.tri & 2) khi = std::min(khi, m0 + BM);
      if (g.tri & 4) khi = std::min(khi, n0 + BN);
      if (khi > klo) fl += 2.0 * std::min(BM, g.m - m0) * std::min(BN, g.n - n0) * (double)(khi - klo);
    }
  return fl * g.batch;
}

hipError_t gemm_f64(const GemmArgs& g, hipStream_t st) { return gemm_f64_cfg(g, st, 0, 0); }

// ---- work lists for products with uneven tiles ----------------------------------------------------------
// Workgroup i of a launch runs on XCD i mod 8, so a grid in tile order gives each XCD whatever tiles land on
// it: with a lower-only result or triangular operands (work per tile from the full K down to one slice) some
// XCDs get several times the work of others.  The work list deals the (tile, K slice) units, longest first,
// each to the XCD with the least work so far, and lays them out so that entry i belongs to XCD i mod 8.  One
// list per shape, built on first use and kept for the life of the process (a few KB each).
constexpr int kXcds = 8;
struct UnitKey {
  int dev, m, n, k, tri, lower, kchunk;
  bool operator<(const UnitKey& o) const {
    return std::tie(dev, m, n, k, tri, lower, kchunk) < std::tie(o.dev, o.m, o.n, o.k, o.tri, o.lower, o.kchunk);
  }
};
struct UnitList {
  int* dev = nullptr;
  int len = 0;
};
static std::mutex g_units_mu;
static std::map<UnitKey, UnitList>* g_units = nullptr;
// The lists live in one device pool reserved outside any solve (gemm_reserve, from context creation): building
// a list in the middle of a solve then needs no allocation and no copy on the legacy stream, which could
// disturb a graph capture running on another thread's stream.
constexpr size_t kUnitPool = size_t(1) << 20;  // ints per device
constexpr int kMaxDevices = 64;
static int* g_unit_pool[kMaxDevices] = {};
static size_t g_unit_used[kMaxDevices] = {};

// *out = null when no list can be built (pool full, or the stream is being captured): the caller then runs
// the plain tile grid.
static hipError_t unit_list(const GemmArgs& g, int kchunk, hipStream_t st, const UnitList** out) {
  int dev = 0;
  KOT_HIP_TRY(hipGetDevice(&dev));
  const UnitKey key{dev, g.m, g.n, g.k, g.tri, g.lower, kchunk};
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDevices) return hipSuccess;
  std::lock_guard<std::mutex> lk(g_units_mu);
  if (!g_units) g_units = new std::map<UnitKey, UnitList>();
  auto it = g_units->find(key);
  if (it != g_units->end()) {
    *out = &it->second;
    return hipSuccess;
  }
  if (!g_unit_pool[dev]) return hipSuccess;
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  KOT_HIP_TRY(hipStreamIsCapturing(st, &cap));
  if (cap != hipStreamCaptureStatusNone) return hipSuccess;
  struct U { int code, work; };
  std::vector<U> us;
  for (int m0 = 0; m0 < g.m; m0 += BM)
    for (int n0 = 0; n0 < g.n; n0 += BN) {
      if (g.lower && n0 > m0 + BM - 1) continue;
      int klo = 0, khi = g.k;
      if (g.tri & 1) klo = std::max(klo, m0);
      if (g.tri & 8) klo = std::max(klo, n0);
      if (g.tri & 2) khi = std::min(khi, m0 + BM);
      if (g.tri & 4) khi = std::min(khi, n0 + BN);
      klo &= ~(BK - 1);
      const int code = ((m0 / BM) << 16) | ((n0 / BN) << 8);
      if (khi <= klo) {  // an empty K range still writes its tile (alpha * 0 + beta * C) when not split
        if (kchunk >= g.k) us.push_back({code, 1});
        continue;
      }
      for (int sp = klo / kchunk; sp * kchunk < khi; ++sp) {
        const int w = std::min(khi, sp * kchunk + kchunk) - std::max(klo, sp * kchunk);
        us.push_back({code | sp, w + BK});  // + a slice's fixed cost
      }
    }
  std::stable_sort(us.begin(), us.end(), [](const U& a, const U& b) { return a.work > b.work; });
  std::vector<std::vector<int>> bins(kXcds);
  std::vector<long long> load(kXcds, 0);
  for (const U& u : us) {
    int b = 0;
    for (int x = 1; x < kXcds; ++x)
      if (load[x] < load[b]) b = x;
    bins[b].push_back(u.code);
    load[b] += u.work;
  }
  size_t rows = 0;
  for (const auto& b : bins) rows = std::max(rows, b.size());
  std::vector<int> host(rows * kXcds, -1);
  for (int x = 0; x < kXcds; ++x)
    for (size_t r = 0; r < bins[x].size(); ++r) host[r * kXcds + x] = bins[x][r];
  if (g_unit_used[dev] + host.size() > kUnitPool) return hipSuccess;
  UnitList ul;
  ul.len = (int)host.size();
  ul.dev = g_unit_pool[dev] + g_unit_used[dev];
  KOT_HIP_TRY(hipMemcpyAsync(ul.dev, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice, st));
  KOT_HIP_TRY(hipStreamSynchronize(st));  // host is a local vector
  g_unit_used[dev] += host.size();
  *out = &((*g_units)[key] = ul);
  return hipSuccess;
}

hipError_t gemm_reserve() {
  int dev = 0;
  KOT_HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return hipSuccess;  // such a device runs without work lists
  std::lock_guard<std::mutex> lk(g_units_mu);
  if (g_unit_pool[dev]) return hipSuccess;
  return hipMalloc(&g_unit_pool[dev], kUnitPool * sizeof(int));
}

hipError_t gemm_f64_cfg(const GemmArgs& g, hipStream_t st, int waves, int splits_req) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return hipSuccess;
  if (g.k <= 0) {  // C = beta C
    // handled by a k=1 launch with alpha = 0 would read A; do it explicitly instead
    return hipErrorInvalidValue;
  }
  if (g.D && (g.batch != 1 || g.lower || g.mirror || !g.y)) return hipErrorInvalidValue;
  if (g.n == 1 && g.batch == 1 && !g.transa && !g.D) {
    // x[c] = op(B)[c][0]: B[c*ldb] (k x 1) or B[c] (1 x k, transposed)
    const int incx = g.transb ? 1 : g.ldb;
    Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
    if (pf) pf->begin(st, PROF_GEMV_F64, 2.0 * g.m * (double)g.k,
                      8.0 * ((double)g.m * g.k + g.k + (g.beta != 0.0 ? 2.0 : 1.0) * g.m));
    hipLaunchKernelGGL(gemv_f64_kernel, dim3((unsigned)((g.m + 3) / 4)), dim3(256), 0, st, g.m, g.k, g.alpha, g.A,
                       g.lda, g.s, g.B, incx, g.beta, g.C, g.ldc);
    if (pf) pf->end(st);
    return hipGetLastError();
  }
  if (waves == 0 && splits_req == 0 && g.batch == 1 && !g.tri && (g.m == 1 || g.k == 1)) {
    Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
    if (g.m == 1 && !g.lower && !g.mirror) {
      // row vector times a matrix: a matrix-vector product, bound by reading op(B)
      const int inca = g.transa ? g.lda : 1;
      const int ks = std::max(1, std::min(kRowvecMaxSlices, (g.k + 15) / 16));
      const bool ws_ok = g_gemm_ws && (size_t)ks * g.n <= g_gemm_ws_cap;
      const bool dot_ok = g.transb && g.k <= kRowvecMaxK;
      if (pf && (dot_ok || (!g.transb && ws_ok)))
        pf->begin(st, PROF_GEMV_F64, 2.0 * g.n * (double)g.k,
                  8.0 * ((double)g.n * g.k + g.k + (g.D ? 3.0 : (g.beta != 0.0 ? 2.0 : 1.0)) * g.n));
      if (dot_ok) {
        hipLaunchKernelGGL(rowvec_dot_kernel, dim3((unsigned)((g.n + 3) / 4)), dim3(256), 0, st, g.n, g.k, g.A, inca,
                           g.s, g.B, g.ldb, g.alpha, g.beta, g.C, g.D, g.dalpha, g.dbeta, g.y);
        if (pf) pf->end(st);
        return hipGetLastError();
      }
      if (!g.transb && ws_ok) {
        const int kc = (g.k + ks - 1) / ks;
        hipLaunchKernelGGL(rowvec_colsum_kernel, dim3((unsigned)((g.n + 63) / 64), (unsigned)ks), dim3(256), 0, st,
                           g.n, g.k, kc, g.A, inca, g.s, g.B, g.ldb, g_gemm_ws);
        KOT_HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(rowvec_final_kernel, dim3((unsigned)((g.n + 255) / 256)), dim3(256), 0, st, g.n, ks,
                           (const double*)g_gemm_ws, g.alpha, g.beta, g.C, g.D, g.dalpha, g.dbeta, g.y);
        if (pf) pf->end(st);
        return hipGetLastError();
      }
    } else if (g.k == 1 && !g.D && (!g.mirror || (g.lower && g.m == g.n && g.beta == 0.0))) {
      // outer product: bound by writing C
      const int inca = g.transa ? 1 : g.lda;  // op(A)_i0
      const int incb = g.transb ? g.ldb : 1;  // op(B)_0j
      if (pf) pf->begin(st, PROF_GEMV_F64, 2.0 * g.m * (double)g.n, 8.0 * (g.beta != 0.0 ? 2.0 : 1.0) * g.m * g.n);
      hipLaunchKernelGGL(rank1_kernel, dim3((unsigned)((g.n + 63) / 64), (unsigned)((g.m + 3) / 4)), dim3(256), 0, st,
                         g.m, g.n, g.alpha, g.A, inca, g.s, g.B, incb, g.beta, g.C, g.ldc, g.lower, g.mirror);
      if (pf) pf->end(st);
      return hipGetLastError();
    }
  }
  const int tiles = ((g.n + BN - 1) / BN) * ((g.m + BM - 1) / BM) * g.batch;
  // 16 waves per workgroup: measured fastest on every solver shape (four waves per SIMD at one tile per CU)
  if (waves == 0) waves = 16;
  int splits = 1;
  int kchunk = g.k;
  if (splits_req > 0) {
    splits = std::min(splits_req, std::max(1, g.k / BK));
  } else {
    // K split: aim for `target` workgroups (one per CU by default; per size bucket from the autotuner's table)
    int target = g_gemm_tune ? g_gemm_tune[gemm_tune_bucket(std::max(g.m, g.n))] : 256;
    const int computed = g.lower ? (tiles + ((g.n + BN - 1) / BN) * g.batch) / 2 : tiles;
    if (g.tri || g.lower) {
      // uneven or halved work: count the (tile, K slice) work units of a slice width, and take the widest
      // slice (a multiple of BK, at least 64) that yields 1.5 x target units, so that the longest K ranges
      // are cut into pieces and every CU gets work
      auto units = [&](int kc) {
        long long u = 0;
        for (int m0 = 0; m0 < g.m; m0 += BM)
          for (int n0 = 0; n0 < g.n; n0 += BN) {
            if (g.lower && n0 > m0 + BM - 1) continue;
            int klo = 0, khi = g.k;
            if (g.tri & 1) klo = std::max(klo, m0);
            if (g.tri & 8) klo = std::max(klo, n0);
            if (g.tri & 2) khi = std::min(khi, m0 + BM);
            if (g.tri & 4) khi = std::min(khi, n0 + BN);
            klo &= ~(BK - 1);
            if (khi > klo) u += (khi - 1) / kc - klo / kc + 1;
          }
        return u * g.batch;
      };
      if (target > 0 && g.k >= 128) {
        const long long want = (long long)target * 3 / 2;
        int kc = (g.k + BK - 1) / BK * BK;
        while (kc > 64 && units(kc) < want) kc = std::max(64, (kc / 2 + BK - 1) / BK * BK);
        kchunk = kc;
        splits = (g.k + kchunk - 1) / kchunk;
      }
    } else if (target > 0 && computed < target && g.k >= 128) {
      splits = (target + computed - 1) / computed;
      splits = std::min(splits, std::min(16, g.k / 64));
    }
  }
  if (splits > 1) {
    const size_t need = (size_t)splits * g.batch * (size_t)g.m * g.n;
    if (!g_gemm_ws || need > g_gemm_ws_cap) {
      splits = 1;
      kchunk = g.k;
    }
  }
  if (splits > 1 && kchunk == g.k) {
    kchunk = ((g.k + splits - 1) / splits + BK - 1) / BK * BK;
    splits = (g.k + kchunk - 1) / kchunk;
  }
  dim3 grid((g.n + BN - 1) / BN, (g.m + BM - 1) / BM, g.batch * splits);
  const int* units = nullptr;
  if ((g.tri || g.lower) && g.batch == 1 && g.m <= 64 * BM && g.n <= 64 * BN && splits <= 255) {
    const UnitList* ul = nullptr;
    KOT_HIP_TRY(unit_list(g, splits > 1 ? kchunk : g.k, st, &ul));
    if (ul) {
      units = ul->dev;
      grid = dim3(ul->len, 1, 1);
    }
  }
  const bool sc = g.s != nullptr;
  Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
  // work of the product (2mnk flops, less the skipped tiles and K ranges); bytes = each operand and C once
  if (pf) pf->begin(st, PROF_GEMM_F64, gemm_work_flops(g),
                    8.0 * g.batch * ((double)g.m * g.k + (double)g.k * g.n + (g.beta != 0.0 ? 2.0 : 1.0) * g.m * g.n));
  if (g.D && (!g_gemm_ws || (size_t)((g.m + BM - 1) / BM) * splits * g.n > g_gemm_ws_cap))
    return hipErrorInvalidValue;
  double* part = (splits > 1 || g.D) ? g_gemm_ws : nullptr;
  bool launched = false;
#define KOT_GEMM_CASE(TA, TB, SC_, FM, FN)                                                                       \
  if (!launched && g.transa == TA && g.transb == TB && sc == SC_ && waves == (4 / FM) * (4 / FN)) {               \
    hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, SC_, FM, FN>), grid, dim3(64 * (4 / FM) * (4 / FN)), 0, st, g,    \
                       splits, kchunk, part, units);                                                               \
    launched = true;                                                                                               \
  }
#define KOT_GEMM_WAVES(FM, FN)                                                                                     \
  KOT_GEMM_CASE(0, 0, false, FM, FN) KOT_GEMM_CASE(0, 1, false, FM, FN) KOT_GEMM_CASE(1, 0, false, FM, FN)         \
  KOT_GEMM_CASE(1, 1, false, FM, FN) KOT_GEMM_CASE(0, 0, true, FM, FN) KOT_GEMM_CASE(0, 1, true, FM, FN)           \
  KOT_GEMM_CASE(1, 0, true, FM, FN) KOT_GEMM_CASE(1, 1, true, FM, FN)
  KOT_GEMM_WAVES(2, 2) KOT_GEMM_WAVES(1, 2) KOT_GEMM_WAVES(1, 1)
#undef KOT_GEMM_WAVES
#undef KOT_GEMM_CASE
  if (!launched) return hipErrorInvalidValue;
  if (g.D) {
    hipLaunchKernelGGL(coldot_final_kernel, dim3((g.n + 63) / 64), dim3(256), 0, st, g, splits, kchunk,
                       (const double*)part);
  } else if (splits > 1) {
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((g.n + BN - 1) / BN, (g.m + RS - 1) / RS, g.batch), dim3(256), 0,
                       st, g, splits, kchunk, (const double*)part);
  }
  if (pf) pf->end(st);
  return hipGetLastError();
}

hipError_t gemv2(int m, const double* Q, double a, const double* K2, double b, const double* v, double c, double* y,
                 hipStream_t st) {
  hipLaunchKernelGGL(gemv2_f64_kernel, dim3((unsigned)((m + 3) / 4)), dim3(256), 0, st, m, Q, a, K2, b, v, c, y);
  return hipGetLastError();
}

hipError_t diag_dot(int r0, int r1, int n, double alpha, const double* A, int lda, const double* B, int ldb,
                    double beta, double* y, double* part, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  dim3 g1((n + 63) / 64, kDiagParts);
  hipLaunchKernelGGL(diag_dot_part, g1, dim3(256), 0, st, r0, r1, n, A, lda, B, ldb, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(diag_dot_final, dim3((n + 255) / 256), dim3(256), 0, st, n, alpha, beta, part, y);
  return hipGetLastError();
}

}  // namespace kot
