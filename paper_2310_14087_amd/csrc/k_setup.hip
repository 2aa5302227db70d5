// Dual data of Eq. (3.4) (Section 3): Gaussian Gram matrices at the filling points, mean embeddings, q^2, z,
// and the upper Cholesky factor R of K + eps I.  FP64 vector ALU; every reduction has a fixed order.
#include "kot_internal.h"

namespace kot {
namespace {

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Q = K_X + K_Y, K = K_X o K_Y (the Gaussian on the concatenated point) on one 32 x 32 tile pair (bi <= bj) per
// workgroup: both results are symmetric, so each pair of exponentials is evaluated once and the tile of the
// lower triangle goes out transposed through LDS as row segments ((a - b)^2 = (b - a)^2 exactly, so the
// mirrored entry is the one a direct evaluation would give).
__global__ __launch_bounds__(256) void gram_sym_kernel(int l, int d, const double* __restrict__ xf,
                                                       const double* __restrict__ yf, double inv2s2,
                                                       double* __restrict__ Q, double* __restrict__ K) {
  __shared__ double tq[32][33], tk[32][33];
  const int nt = (l + 31) / 32;
  int u = blockIdx.x, bi = 0;
  while (u >= nt - bi) {  // row bi of the upper triangle holds nt - bi tiles
    u -= nt - bi;
    ++bi;
  }
  const int bj = bi + u;
  const int t = threadIdx.x, tc = t & 31, tr = t >> 5;
  const int j = bj * 32 + tc;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ii = tr + 8 * q, i = bi * 32 + ii;
    if (i < l && j < l) {
      double dx = 0.0, dy = 0.0;
      for (int k = 0; k < d; ++k) {
        const double a = xf[(long long)i * d + k] - xf[(long long)j * d + k];
        const double b = yf[(long long)i * d + k] - yf[(long long)j * d + k];
        dx += a * a;
        dy += b * b;
      }
      const double kx = exp(-dx * inv2s2), ky = exp(-dy * inv2s2);
      Q[(long long)i * l + j] = kx + ky;
      K[(long long)i * l + j] = kx * ky;
      tq[ii][tc] = kx + ky;
      tk[ii][tc] = kx * ky;
    }
  }
  if (bi == bj) return;  // uniform per workgroup
  __syncthreads();
  const int i2 = bi * 32 + tc;  // column of the transposed write
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int jj = tr + 8 * q, j2 = bj * 32 + jj;
    if (i2 < l && j2 < l) {
      Q[(long long)j2 * l + i2] = tq[tc][jj];
      K[(long long)j2 * l + i2] = tk[tc][jj];
    }
  }
}

// w[i] = (1/n) sum_j exp(-|s_j - p_i|^2 inv2s2): 4 points per workgroup, samples strided over 256 threads,
// then a fixed tree reduction.
constexpr int EPT = 4;
__global__ __launch_bounds__(256) void embed_kernel(int n, int l, int d, const double* __restrict__ s, const double* __restrict__ p,
                                                     double inv2s2, double* __restrict__ w) {
  __shared__ double red[EPT][256];
  __shared__ double pt[EPT][64];
  const int i0 = blockIdx.x * EPT;
  for (int u = threadIdx.x; u < EPT * d && u < EPT * 64; u += 256) {
    const int q = u / d, k = u % d;
    pt[q][k] = (i0 + q < l) ? p[(long long)(i0 + q) * d + k] : 0.0;
  }
  __syncthreads();
  double acc[EPT] = {0.0, 0.0, 0.0, 0.0};
  for (int j = threadIdx.x; j < n; j += 256) {
    double d2[EPT] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < d; ++k) {
      const double v = s[(long long)j * d + k];
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        const double a = v - pt[q][k];
        d2[q] += a * a;
      }
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q) acc[q] += exp(-d2[q] * inv2s2);
  }
#pragma unroll
  for (int q = 0; q < EPT; ++q) red[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
#pragma unroll
      for (int q = 0; q < EPT; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < EPT && i0 + threadIdx.x < l) w[i0 + threadIdx.x] = red[threadIdx.x][0] / (double)n;
}

// Sum of k(x_i, x_j) over the pairs i < j of one 64 x 64 tile pair (I, J), I <= J (symmetry halves the
// work; the diagonal contributes n exactly since k(x, x) = 1).  Both tiles are staged in LDS; lane t of
// wave g takes column j = 64 J + t against rows 64 I + 16 g .. + 15, so the row operands are LDS
// broadcasts.  Workgroups with J < I write a zero partial.  part[I * nt + J]; fixed order throughout.
constexpr int QT = 64;
__global__ __launch_bounds__(256) void gram_pairsum_kernel(int n, int d, const double* __restrict__ x, double inv2s2,
                                                           double* __restrict__ part) {
  __shared__ double xi[QT][QT + 1];   // [row][k]
  __shared__ double xj[QT][QT + 1];   // [k][col]
  __shared__ double red[256];
  const int J = blockIdx.x, I = blockIdx.y, nt = gridDim.x;
  const int t = threadIdx.x;
  if (J < I) {
    if (t == 0) part[(long long)I * nt + J] = 0.0;
    return;
  }
  const int i0 = I * QT, j0 = J * QT;
  for (int u0 = 0; u0 < QT * d; u0 += 4 * 256) {  // four loads per operand in flight per pass
    double vi[4], vj[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = u0 + t + 256 * q, r = u / d, k = u - r * d;
      const bool in = u < QT * d;
      vi[q] = (in && i0 + r < n) ? x[(long long)(i0 + r) * d + k] : 0.0;
      vj[q] = (in && j0 + r < n) ? x[(long long)(j0 + r) * d + k] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = u0 + t + 256 * q, r = u / d, k = u - r * d;
      if (u < QT * d) { xi[r][k] = vi[q]; xj[k][r] = vj[q]; }
    }
  }
  __syncthreads();
  const int c = t & 63, g = t >> 6;
  double d2[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) d2[r] = 0.0;
  for (int k = 0; k < d; ++k) {
    const double v = xj[k][c];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const double a = xi[g * 16 + r][k] - v;
      d2[r] += a * a;
    }
  }
  const int gj = j0 + c;
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gi = i0 + g * 16 + r;
    if (gi < gj && gj < n) acc += exp(-d2[r] * inv2s2);
  }
  red[t] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) red[t] += red[t + h];
    __syncthreads();
  }
  if (t == 0) part[(long long)I * nt + J] = red[0];
}

// out[0] = (n + 2 sum(part[0..np))) / n^2
__global__ __launch_bounds__(256) void pairsum_final_kernel(int n, int np, const double* __restrict__ part, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < np; j += 256) acc += part[j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = ((double)n + 2.0 * red[0]) / ((double)n * (double)n);
}

__global__ void z_kernel(int l, int d, const double* __restrict__ xf, const double* __restrict__ yf, const double* __restrict__ wmu,
                         const double* __restrict__ wnu, double lam2, double* __restrict__ z, double* __restrict__ wsum) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  double c = 0.0;
  for (int k = 0; k < d; ++k) {
    const double a = xf[(long long)i * d + k] - yf[(long long)i * d + k];
    c += a * a;
  }
  const double ws = wmu[i] + wnu[i];
  wsum[i] = ws;
  z[i] = ws - lam2 * c;
}

// ---------------------------------------------------------------------------------------------------------
// Blocked right-looking Cholesky on a working copy W (lower triangle), panel width CB, one launch per panel
// with a one-panel look-ahead.  Launch s factors panel s (columns k0 = s CB ..) and, in the same grid,
// applies the previous panel's L21 to the trailing lower triangle beyond panel s; the previous panel's
// contribution to panel s itself is applied by the panel workgroups just before they factor it.  Panel s
// therefore never waits for the trailing update of step s - 1, which runs beside it.
constexpr int CB = 32;

__device__ __forceinline__ double readlane_f64(double x, int lane) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// ---- the inverse X = L^-1 (lower, CB-blocked) beside the factorization ------------------------------------
// Forward substitution L X = I by block rows: X_rr = L_rr^-1 and X_rj = -L_rr^-1 C_rj, C_rj = sum over
// m = j .. r-1 of L_rm X_mj, accumulated right-looking in X's own storage (zero on entry).  Launch s, where
// block rows <= s - 1 of L are final, finishes row r = s - 1 (adding the m = r - 1 term itself, as the panel
// workgroups do for the factor) and adds the m = s - 2 term to the rows k >= s.  Tiles of 32 x 32 live in the
// four quadrants of the workgroup's LDS array (row stride 2 CB + 1).
#define QT(q, i, k) S[((q) >> 1) * CB + (i)][((q) & 1) * CB + (k)]

// Block (rb, cb) of the l x l row-major M into LDS quadrant q; entries past l read as zero, or as the
// identity when pad_eye (a short last diagonal block).  All loads of a lane in flight together.
__device__ __forceinline__ void load_quad(const double* __restrict__ M, int l, int rb, int cb, int q, bool pad_eye,
                                          double (*S)[2 * CB + 1], int t) {
  double v[CB * CB / 64];
#pragma unroll
  for (int e = 0; e < CB * CB / 64; ++e) {
    const int u = t + 64 * e, i = u >> 5, k = u & 31;
    v[e] = M[(long long)min(rb * CB + i, l - 1) * l + min(cb * CB + k, l - 1)];
  }
#pragma unroll
  for (int e = 0; e < CB * CB / 64; ++e) {
    const int u = t + 64 * e, i = u >> 5, k = u & 31;
    const bool in = rb * CB + i < l && cb * CB + k < l;
    QT(q, i, k) = in ? v[e] : ((pad_eye && i == k) ? 1.0 : 0.0);
  }
}

// Launch s, block (r, j), j <= r, r = s - 1: X_rj from C_rj + L_{r,r-1} X_{r-1,j} (j < r) or the identity (j = r).
__device__ void inv_row_block(int l, int r, int j, const double* __restrict__ W, double* __restrict__ Y,
                              double (*S)[2 * CB + 1], double* invd, int t) {
  load_quad(W, l, r, r, 0, true, S, t);             // L_rr
  if (j < r) {
    load_quad(W, l, r, r - 1, 1, false, S, t);      // L_{r,r-1}
    load_quad(Y, l, r - 1, j, 2, false, S, t);      // X_{r-1,j}
    load_quad(Y, l, r, j, 3, false, S, t);          // C_rj
  }
  __syncthreads();
  if (t < CB) invd[t] = 1.0 / QT(0, t, t);
  if (j < r) {
    // B = -(C_rj + L_{r,r-1} X_{r-1,j}) on the matrix cores (operand lane L: A[L%16][L/16], B[L/16][L%16];
    // accumulator lane L: D[L/16 + 4 v][L%16]); each lane rewrites the entries of C it read
    const int r16 = t & 15, k4 = t >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[rb][cb][v] = QT(3, rb * 16 + k4 + 4 * v, cb * 16 + r16);
    double fa[2][CB / 4], fb[2][CB / 4];
#pragma unroll
    for (int ks = 0; ks < CB / 4; ++ks)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        fa[h][ks] = QT(1, h * 16 + r16, ks * 4 + k4);
        fb[h][ks] = QT(2, ks * 4 + k4, h * 16 + r16);
      }
#pragma unroll
    for (int ks = 0; ks < CB / 4; ++ks)
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[rb][ks], fb[cb][ks], acc[rb][cb], 0, 0, 0);
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int v = 0; v < 4; ++v) QT(3, rb * 16 + k4 + 4 * v, cb * 16 + r16) = -acc[rb][cb][v];
  }
  __syncthreads();
  if (t >= CB) return;
  // L_rr x = b for column t of B (or of the identity): once x_q is final it leaves every later entry
  double x[CB];
#pragma unroll
  for (int i = 0; i < CB; ++i) x[i] = (j < r) ? QT(3, i, t) : (i == t ? 1.0 : 0.0);
#pragma unroll
  for (int q = 0; q < CB; ++q) {
    x[q] *= invd[q];
#pragma unroll
    for (int i = q + 1; i < CB; ++i) x[i] = fma(-QT(0, i, q), x[q], x[i]);
#pragma unroll
    for (int i = q; i < CB; ++i) asm volatile("" : "+v"(x[i]));  // each step in order (else it spills)
  }
  const int col = j * CB + t;
  if (col < l)
#pragma unroll
    for (int i = 0; i < CB; ++i)
      if (r * CB + i < l) Y[(long long)(r * CB + i) * l + col] = x[i];
}

// Launch s, tile u of the rows k >= s and columns j <= m = s - 2: C_kj += L_km X_mj.
__device__ void inv_update_block(int l, int s, int u, const double* __restrict__ W, double* __restrict__ Y,
                                 double (*S)[2 * CB + 1], int t) {
  const int m = s - 2;
  const int k = s + u / (m + 1), j = u % (m + 1);
  const int ri = (t >> 3) * 4, ci = (t & 7) * 4;
  double cv[4][4];
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) cv[p][q] = Y[(long long)min(k * CB + ri + p, l - 1) * l + min(j * CB + ci + q, l - 1)];
  load_quad(W, l, k, m, 0, false, S, t);  // L_km
  load_quad(Y, l, m, j, 1, false, S, t);  // X_mj
  __syncthreads();
#pragma unroll 8
  for (int q = 0; q < CB; ++q) {
    double av[4], bv[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      av[p] = QT(0, ri + p, q);
      bv[p] = QT(1, q, ci + p);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int e = 0; e < 4; ++e) cv[p][e] = fma(av[p], bv[e], cv[p][e]);
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int rr = k * CB + ri + p;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int cc = j * CB + ci + e;
      if (rr < l && cc < l) Y[(long long)rr * l + cc] = cv[p][e];
    }
  }
}
#undef QT

// Panel workgroups (one wavefront each): lanes 0..31 hold the rows of the CB x CB diagonal block (every
// workgroup factors it; workgroup 0 writes it back and reports a non-positive pivot through info), lanes
// 32..63 the CB panel rows k0 + nb + 32 b ..; the right-looking factorization of this 64-row tall panel
// turns the lower rows into L21 with no separate triangular solve.  At step j the pivot reaches every lane
// through v_readlane (the next pivot is formed on its own lane ahead of the rest of the update) and the new
// column L_.j through LDS.
// Update workgroups: the 32 x 32 tiles (tr >= tc) of W[k0 + CB.., k0 + CB..] get -= L_r L_c^T over the
// previous panel's columns, staged in LDS; each lane accumulates a 4 x 4 block.
__global__ __launch_bounds__(64) void chol_step_kernel(int l, int k0, int nb, int npb, int ntiles, int nir,
                                                       double* __restrict__ W, int* info, double* __restrict__ Y) {
  __shared__ double S[64][2 * CB + 1];  // panel: the workgroup's rows over both panels; update: the two L tiles
  __shared__ double colb[2][CB];
  double (*Lb)[2 * CB + 1] = S;
  double (*Lc)[2 * CB + 1] = S + CB;
  const int t = threadIdx.x;
  const int kp = k0 - CB;  // first column of the previous panel (< 0: none)
  const int bid = (int)blockIdx.x;
  if (bid >= npb + ntiles) {
    // ---- the inverse X = L^-1, one block row behind the factorization (launch s: row s - 1)
    const int s = k0 / CB;
    if (bid < npb + ntiles + nir) inv_row_block(l, s - 1, bid - npb - ntiles, W, Y, S, colb[0], t);
    else inv_update_block(l, s, bid - npb - ntiles - nir, W, Y, S, t);
    return;
  }
  if (bid >= npb) {
    // ---- trailing update with the previous panel: tile u of the lower triangle beyond panel s
    int u = bid - npb, tr = 0;
    while (u > tr) { u -= tr + 1; ++tr; }
    const int tc = u;
    const int o = k0 + CB, R0 = o + CB * tr, C0 = o + CB * tc;
    // stage L[R0.., kp..] and L[C0.., kp..] (rows past l read as zero), and fetch this lane's 4 x 4 block of the
    // tile: all loads of a lane in flight together, from clamped (in-bounds) addresses
    const int ri = (t >> 3) * 4, ci = (t & 7) * 4;
    double cv[4][4];
    {
      double vb[CB * CB / 64], vc[CB * CB / 64];
#pragma unroll
      for (int q = 0; q < CB * CB / 64; ++q) {
        const int e = t + 64 * q, r = e >> 5, k = e & 31;
        vb[q] = W[(long long)min(R0 + r, l - 1) * l + kp + k];
        vc[q] = W[(long long)min(C0 + r, l - 1) * l + kp + k];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          cv[p][q] = W[(long long)min(R0 + ri + p, l - 1) * l + min(C0 + ci + q, l - 1)];
#pragma unroll
      for (int q = 0; q < CB * CB / 64; ++q) {
        const int e = t + 64 * q, r = e >> 5, k = e & 31;
        Lb[r][k] = (R0 + r < l) ? vb[q] : 0.0;
        Lc[r][k] = (C0 + r < l) ? vc[q] : 0.0;
      }
    }
    __syncthreads();
    double acc[4][4] = {};
#pragma unroll 8
    for (int k = 0; k < CB; ++k) {
      double av[4], bv[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        av[p] = Lb[ri + p][k];
        bv[p] = Lc[ci + p][k];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(av[p], bv[q], acc[p][q]);
    }
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int r = R0 + ri + p;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cc = C0 + ci + q;
        if (r < l && cc <= r) W[(long long)r * l + cc] = cv[p][q] - acc[p][q];  // cc <= r < l
      }
    }
    return;
  }
  // ---- panel s
  const bool diag = t < CB;
  const int row = diag ? k0 + t : k0 + nb + (int)blockIdx.x * CB + (t - CB);
  const bool live = diag ? t < nb : row < l;
  // stage the 64 rows of this workgroup over the column window [k0 - CB, k0 + CB) (the previous panel, then
  // this one) in LDS: each load instruction reads one row segment, lane t column t of the window
  {
    const int w0 = kp >= 0 ? kp : k0;
    const int wn = kp >= 0 ? 2 * CB : CB;
    const int wc = min(wn, k0 + nb - w0);  // columns of the window inside the matrix
    // clamped addresses keep every load in bounds without a branch; the entries they fill for rows past l or
    // columns past the window are finite copies of real entries, and nothing that is stored depends on them
    const int tc = min(t, wc - 1);
    double v[64];
#pragma unroll
    for (int q = 0; q < 64; ++q) {
      const int r = q < CB ? k0 + q : k0 + nb + (int)blockIdx.x * CB + (q - CB);
      v[q] = W[(long long)min(r, l - 1) * l + w0 + tc];
    }
#pragma unroll
    for (int q = 0; q < 64; ++q) S[q][t] = v[q];
  }
  __syncthreads();
  if (kp >= 0) {
    // the previous panel's contribution to this panel's columns, S[r][CB + c] -= sum_k S[r][k] S[c][k] (rows
    // c < CB of S are the diagonal block's), as a 64 x 32 x 32 product on the matrix cores: operand lane L
    // supplies A[L%16][L/16] and B[L/16][L%16], the accumulator lane L holds D[L/16 + 4 v][L%16].  With
    // B = A^T of the diagonal rows, both operands come from the same fragments.  Rows that are not live
    // are updated too: they are replaced (diagonal padding) or never stored.
    const int r16 = t & 15, k4 = t >> 4;
    double f[4][CB / 4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int ks = 0; ks < CB / 4; ++ks) f[rb][ks] = S[rb * 16 + r16][ks * 4 + k4];
    dbl4 acc[4][2];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = dbl4{0.0, 0.0, 0.0, 0.0};
    // (block rb = 0, cb = 1 lies above the diagonal of the diagonal block: not needed)
#pragma unroll
    for (int ks = 0; ks < CB / 4; ++ks)
#pragma unroll
      for (int rb = 0; rb < 4; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
          if (rb > 0 || cb == 0)
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(f[rb][ks], f[cb][ks], acc[rb][cb], 0, 0, 0);
#pragma unroll
    for (int rb = 0; rb < 4; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        if (rb > 0 || cb == 0)
#pragma unroll
          for (int v = 0; v < 4; ++v) S[rb * 16 + k4 + 4 * v][CB + cb * 16 + r16] -= acc[rb][cb][v];
    __syncthreads();
  }
  const int ca = kp >= 0 ? CB : 0;  // column of this panel inside the staged window
  double a[CB];
#pragma unroll
  for (int c = 0; c < CB; ++c) {
    const double v = S[t][ca + c];
    a[c] = diag ? (live ? ((c <= t) ? v : 0.0) : ((t == c) ? 1.0 : 0.0)) : v;  // short block: identity pad
  }
  // Right-looking factorization of the 64 x CB panel, pipelined: step j's update reaches columns j + 1 and
  // j + 2 at once, through the L entries of rows k0 + j + 1 and k0 + j + 2 read from their lanes; the rest of
  // it (columns >= j + 3, new column through LDS) is applied during step j + 1, so the LDS round trip and
  // that bulk of FMAs overlap the next pivot's chain.  Every column has all earlier steps' terms before it
  // becomes a pivot column.
  unsigned badmask = 0;  // bit j: the pivot of step j was not a positive normal number
  double pnext = readlane_f64(a[0], 0);
  double lprev = 0.0;  // L(row, k0 + j - 1)
  double cbuf[CB];     // L(k0 + c, k0 + j - 1) for c >= j + 2, read from LDS in the previous step
#pragma unroll
  for (int c = 0; c < CB; ++c) cbuf[c] = 0.0;
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    double piv = pnext;
    // a valid pivot is a positive normal number: high word in [0x00100000, 0x7ff00000) (a scalar test)
    const unsigned hw = (unsigned)((unsigned long long)__double_as_longlong(piv) >> 32);
    if (hw - 0x00100000u >= 0x7fe00000u) {  // recorded, then replaced by 1
      badmask |= 1u << j;
      piv = 1.0;
    }
    asm volatile("" : "+v"(badmask));  // kept in step (left to itself the compiler defers it past the loop)
    // 1/sqrt(piv): hardware estimate y0 refined by one third-order step y0 (1 + e/2 + 3 e^2/8), e = 1 - piv y0^2
    const double y0 = __builtin_amdgcn_rsq(piv);
    const double e = fma(-piv * y0, y0, 1.0);
    const double rdj = fma(y0 * e, fma(0.375, e, 0.5), y0);
    const double dj = piv * rdj;
    const double lij = a[j] * rdj;  // L_ij on rows below j
    if (diag) colb[j & 1][t] = lij;
    if (j + 1 < CB) {
      a[j + 1] = fma(-lij, readlane_f64(lij, j + 1), a[j + 1]);
      pnext = readlane_f64(a[j + 1], j + 1);
    }
    if (j + 2 < CB) a[j + 2] = fma(-lij, readlane_f64(lij, j + 2), a[j + 2]);
    // the bulk of step j - 1
    if (j >= 1)
#pragma unroll
      for (int c = j + 2; c < CB; ++c) a[c] = fma(-lprev, cbuf[c], a[c]);
    __builtin_amdgcn_wave_barrier();  // (one wavefront: LDS operations complete in issue order)
#pragma unroll
    for (int c = j + 3; c < CB; ++c) cbuf[c] = colb[j & 1][c];
    lprev = lij;
    a[j] = (diag && t == j) ? dj : lij;
#pragma unroll
    for (int c = j + 1; c < CB; ++c) asm volatile("" : "+v"(a[c]));  // keep each update inside its step
  }
  if (blockIdx.x == 0 && t == 0) {
    const unsigned m = badmask & (nb >= 32 ? ~0u : ((1u << nb) - 1u));
    if (m) atomicCAS(info, 0, k0 + __ffs((int)m));  // the first non-positive pivot, 1-based
  }
  // stores: lane t writes its row of the panel (the diagonal block, zeros above the diagonal, from
  // workgroup 0 only); the column offsets are immediates of the store instructions
  if (diag) {
    if (blockIdx.x == 0 && live)
#pragma unroll
      for (int c = 0; c < CB; ++c)
        if (c < nb) W[(long long)row * l + k0 + c] = (c <= t) ? a[c] : 0.0;
  } else if (live) {
#pragma unroll
    for (int c = 0; c < CB; ++c) W[(long long)row * l + k0 + c] = a[c];
  }
}

__global__ void copy_jitter_kernel(int l, const double* __restrict__ A, double eps, double* __restrict__ W,
                                   int* __restrict__ info, double* __restrict__ Y) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u == 0) *info = 0;
  if (u >= (long long)l * l) return;
  if (Y) Y[u] = 0.0;
  const int i = (int)(u / l), j = (int)(u % l);
  W[u] = A[u] + ((i == j) ? eps : 0.0);
}

// R[i][j] = L[j][i] for j >= i, 0 below the diagonal.
__global__ void lower_to_upper_kernel(int l, const double* __restrict__ L, double* __restrict__ R) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  R[u] = (j >= i) ? L[(long long)j * l + i] : 0.0;
}

// ---------------------------------------------------------------------------------------------------------
// Y = R^{-1} for upper-triangular R by recursive doubling: all TRB x TRB diagonal blocks are inverted at
// once, then adjacent inverted blocks of width b merge into width 2b through
//   Y12 = -Y11 (R12 Y22),
// every merge of one level in a single batched MFMA GEMM pair.
constexpr int TRB = 32;

// Inverse of the diagonal block starting at r0 = TRB * blockIdx.x (upper triangular); thread c computes
// column c by back substitution.  Entries of the block below its diagonal are written as zero.
__global__ __launch_bounds__(64) void trtri_diag_kernel(int l, const double* __restrict__ R, double* __restrict__ Y) {
  __shared__ double D[TRB][TRB + 1];
  const int r0 = blockIdx.x * TRB;
  const int nb = min(TRB, l - r0);
  {
    double v[TRB * TRB / 64];
#pragma unroll
    for (int q = 0; q < TRB * TRB / 64; ++q) {
      const int u = threadIdx.x + 64 * q, i = u >> 5, j = u & 31;
      v[q] = (i < nb && j < nb) ? R[(long long)(r0 + i) * l + r0 + j] : (i == j ? 1.0 : 0.0);
    }
#pragma unroll
    for (int q = 0; q < TRB * TRB / 64; ++q) {
      const int u = threadIdx.x + 64 * q;
      D[u >> 5][u & 31] = v[q];
    }
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c >= TRB) return;
  double y[TRB];
#pragma unroll
  for (int i = TRB - 1; i >= 0; --i) {
    double v = (i == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = i + 1; k < TRB; ++k) v -= D[i][k] * y[k];
    y[i] = (i <= c) ? v / D[i][i] : 0.0;
  }
  if (c < nb)
#pragma unroll
    for (int i = 0; i < TRB; ++i)
      if (i < nb) Y[(long long)(r0 + i) * l + r0 + c] = y[i];
}

}  // namespace

hipError_t trtri_upper(int l, const double* R, double* Y, double* T, hipStream_t st) {
  KOT_HIP_TRY(mat_fill(l, l, 0.0, Y, l, st));
  hipLaunchKernelGGL(trtri_diag_kernel, dim3((l + TRB - 1) / TRB), dim3(64), 0, st, l, R, Y);
  KOT_HIP_TRY(hipGetLastError());
  for (int b = TRB; b < l; b *= 2) {
    // merges at s = 2b p: left block [s, s+b), right block [s+b, s+b+b2), b2 = min(b, l - s - b)
    const int full = l / (2 * b);                 // merges with b2 == b
    const int s_last = full * 2 * b;              // a ragged merge starts here if s_last + b < l
    for (int pass = 0; pass < 2; ++pass) {
      const int cnt = pass == 0 ? full : ((s_last + b < l) ? 1 : 0);
      if (cnt == 0) continue;
      const int s0 = pass == 0 ? 0 : s_last;
      const int b2 = pass == 0 ? b : l - s_last - b;
      const long long stride = 2LL * b * (l + 1);
      GemmArgs g{};
      g.batch = cnt;
      g.alpha = 1.0; g.beta = 0.0;
      // T12 = R12 Y22  (b x b2)
      g.transa = 0; g.transb = 0; g.m = b; g.n = b2; g.k = b2;
      g.tri = 4;  // Y22 upper triangular
      g.A = R + (long long)s0 * l + s0 + b; g.lda = l; g.sA = stride;
      g.B = Y + (long long)(s0 + b) * l + s0 + b; g.ldb = l; g.sB = stride;
      g.C = T + (long long)s0 * l + s0 + b; g.ldc = l; g.sC = stride;
      KOT_HIP_TRY(gemm_f64(g, st));
      // Y12 = -Y11 T12  (b x b2)
      g.alpha = -1.0; g.m = b; g.n = b2; g.k = b;
      g.tri = 1;  // Y11 upper triangular
      g.A = Y + (long long)s0 * l + s0; g.lda = l; g.sA = stride;
      g.B = T + (long long)s0 * l + s0 + b; g.ldb = l; g.sB = stride;
      g.C = Y + (long long)s0 * l + s0 + b; g.ldc = l; g.sC = stride;
      KOT_HIP_TRY(gemm_f64(g, st));
    }
  }
  return hipSuccess;
}

hipError_t gram_build(int l, int d, const double* xf, const double* yf, double sigma, double* Q, double* K,
                      hipStream_t st) {
  const int nt = (l + 31) / 32;
  hipLaunchKernelGGL(gram_sym_kernel, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, l, d, xf, yf,
                     1.0 / (2.0 * sigma * sigma), Q, K);
  return hipGetLastError();
}

hipError_t mean_embedding(int n, int l, int d, const double* samples, const double* pts, double sigma, double* w,
                          hipStream_t st) {
  if (d > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(embed_kernel, dim3((l + EPT - 1) / EPT), dim3(256), 0, st, n, l, d, samples, pts,
                     1.0 / (2.0 * sigma * sigma), w);
  return hipGetLastError();
}

size_t mean_gram_part_size(int n) {
  const size_t nt = (size_t)((n + QT - 1) / QT);
  return nt * nt;
}

hipError_t mean_gram(int n, int d, const double* x, double sigma, double* out, double* part, hipStream_t st) {
  if (d > QT || n <= 0) return hipErrorInvalidValue;
  const int nt = (n + QT - 1) / QT;
  hipLaunchKernelGGL(gram_pairsum_kernel, dim3(nt, nt), dim3(256), 0, st, n, d, x, 1.0 / (2.0 * sigma * sigma), part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(pairsum_final_kernel, dim3(1), dim3(256), 0, st, n, nt * nt, part, out);
  return hipGetLastError();
}

hipError_t build_z(int l, int d, const double* xf, const double* yf, const double* wmu, const double* wnu, double lam2,
                   double* z, double* wsum, hipStream_t st) {
  hipLaunchKernelGGL(z_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, d, xf, yf, wmu, wnu, lam2, z, wsum);
  return hipGetLastError();
}

hipError_t cholesky_upper(int l, const double* A, double eps, double* R, double* W, int* info, hipStream_t st,
                          double* Linv) {
  const long long nn = (long long)l * l;
  const int eb = (int)((nn + 255) / 256);
  hipLaunchKernelGGL(copy_jitter_kernel, dim3(eb), dim3(256), 0, st, l, A, eps, W, info, Linv);
  KOT_HIP_TRY(hipGetLastError());
  const int nbk = (l + CB - 1) / CB;  // block rows
  for (int s = 0; s <= nbk; ++s) {
    const int k0 = s * CB;
    int npb = 0, ntiles = 0, nir = 0, niu = 0, nb = 0;
    if (s < nbk) {
      nb = (l - k0 < CB) ? (l - k0) : CB;
      const int rest = l - k0 - nb;
      npb = rest > 0 ? (rest + CB - 1) / CB : 1;
      // trailing tiles beyond panel s that the previous panel still has to update
      const int m = (k0 > 0 && l > k0 + CB) ? (l - k0 - CB + CB - 1) / CB : 0;
      ntiles = m * (m + 1) / 2;
    }
    if (Linv) {
      if (s >= 1) nir = s;                                  // row s - 1, blocks 0 .. s - 1
      if (s >= 2 && s < nbk) niu = (nbk - s) * (s - 1);    // rows s .. nbk - 1, blocks 0 .. s - 2
    }
    if (npb + ntiles + nir + niu == 0) continue;
    hipLaunchKernelGGL(chol_step_kernel, dim3(npb + ntiles + nir + niu), dim3(64), 0, st, l, k0, nb, npb, ntiles,
                       nir, W, info, Linv);
    KOT_HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(lower_to_upper_kernel, dim3(eb), dim3(256), 0, st, l, W, R);
  return hipGetLastError();
}

}  // namespace kot
