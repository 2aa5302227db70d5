// Dual data of Eq. (3.4) (Section 3): Gaussian Gram matrices at the filling points, mean embeddings, q^2, z,
// and the upper Cholesky factor R of K + eps I.  FP64 vector ALU; every reduction has a fixed order.
#include "kot_internal.h"

namespace kot {
namespace {

// Q = K_X + K_Y, K = K_X o K_Y (the Gaussian on the concatenated point), one thread per entry.
__global__ __launch_bounds__(256) void gram_kernel(int l, int d, const double* __restrict__ xf, const double* __restrict__ yf,
                                                    double inv2s2, double* __restrict__ Q, double* __restrict__ K) {
  const int j = blockIdx.x * 16 + (threadIdx.x & 15);
  const int i = blockIdx.y * 16 + (threadIdx.x >> 4);
  if (i >= l || j >= l) return;
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

// part[i] = sum_j k(x_i, x_j) for row i (one workgroup per row).
__global__ __launch_bounds__(256) void gram_rowsum_kernel(int n, int d, const double* __restrict__ x, double inv2s2,
                                                           double* __restrict__ part) {
  __shared__ double red[256];
  __shared__ double xi[64];
  const int i = blockIdx.x;
  if (threadIdx.x < d && threadIdx.x < 64) xi[threadIdx.x] = x[(long long)i * d + threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) {
    double d2 = 0.0;
    for (int k = 0; k < d; ++k) {
      const double a = x[(long long)j * d + k] - xi[k];
      d2 += a * a;
    }
    acc += exp(-d2 * inv2s2);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[i] = red[0];
}

__global__ __launch_bounds__(256) void sum_scale_kernel(int n, const double* __restrict__ part, double scale, double* out) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += 256) acc += part[j];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0] * scale;
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
// Blocked right-looking Cholesky on a working copy W (lower triangle), block size CB.
constexpr int CB = 32;

// Factor the diagonal block W[k0:k0+nb, k0:k0+nb] in LDS (one workgroup).
__global__ __launch_bounds__(256) void potrf_diag_kernel(int l, int k0, int nb, double* __restrict__ W, int* info) {
  __shared__ double T[CB][CB + 1];
  for (int u = threadIdx.x; u < nb * nb; u += 256) {
    const int i = u / nb, j = u % nb;
    T[i][j] = W[(long long)(k0 + i) * l + k0 + j];
  }
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    if (threadIdx.x == 0) {
      const double piv = T[j][j];
      if (!(piv > 0.0)) {
        info[0] = k0 + j + 1;
        T[j][j] = 1.0;
      } else {
        T[j][j] = sqrt(piv);
      }
    }
    __syncthreads();
    const double djj = T[j][j];
    for (int i = j + 1 + threadIdx.x; i < nb; i += 256) T[i][j] /= djj;
    __syncthreads();
    // trailing update of the block's lower triangle
    for (int u = threadIdx.x; u < nb * nb; u += 256) {
      const int i = u / nb, c = u % nb;
      if (i > j && c > j && c <= i) T[i][c] -= T[i][j] * T[c][j];
    }
    __syncthreads();
  }
  for (int u = threadIdx.x; u < nb * nb; u += 256) {
    const int i = u / nb, j = u % nb;
    W[(long long)(k0 + i) * l + k0 + j] = (j <= i) ? T[i][j] : 0.0;
  }
}

// Panel: rows r >= k0+nb solve L21 L11^T = A21.  A workgroup stages 64 rows x nb of the panel through LDS
// (coalesced along the row), then each of 64 threads forward-substitutes its row in LDS.
__global__ __launch_bounds__(256) void trsm_panel_kernel(int l, int k0, int nb, double* __restrict__ W) {
  __shared__ double L11[CB][CB + 1];
  __shared__ double P[64][CB + 1];
  const int rbase = k0 + nb + blockIdx.x * 64;
  for (int u = threadIdx.x; u < nb * nb; u += 256) {
    const int i = u / nb, j = u % nb;
    L11[i][j] = W[(long long)(k0 + i) * l + k0 + j];
  }
  for (int u = threadIdx.x; u < 64 * nb; u += 256) {
    const int r = u / nb, j = u % nb;
    P[r][j] = (rbase + r < l) ? W[(long long)(rbase + r) * l + k0 + j] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 64 && rbase + threadIdx.x < l) {
    const int r = threadIdx.x;
    for (int j = 0; j < nb; ++j) {
      double v = P[r][j];
      for (int c = 0; c < j; ++c) v -= P[r][c] * L11[j][c];
      P[r][j] = v / L11[j][j];
    }
  }
  __syncthreads();
  for (int u = threadIdx.x; u < 64 * nb; u += 256) {
    const int r = u / nb, j = u % nb;
    if (rbase + r < l) W[(long long)(rbase + r) * l + k0 + j] = P[r][j];
  }
}

__global__ void copy_jitter_kernel(int l, const double* __restrict__ A, double eps, double* __restrict__ W) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
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
// Y = R^{-1} for upper-triangular R, by row blocks of TRB from the bottom: the block's rows start as identity
// rows, receive -R[blk, below] Y[below, :] from the MFMA GEMM, then are solved against the diagonal block.
constexpr int TRB = 32;

__global__ void eye_rows_kernel(int l, int r0, int nb, double* __restrict__ Y) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)nb * l) return;
  const int r = (int)(u / l), c = (int)(u % l);
  Y[(long long)(r0 + r) * l + c] = (r0 + r == c) ? 1.0 : 0.0;
}

// Y[r0:r0+nb, c] <- R_dd^{-1} Y[r0:r0+nb, c] for every column c (R_dd = R[r0:r0+nb, r0:r0+nb] upper).
__global__ __launch_bounds__(256) void trsv_block_kernel(int l, int r0, int nb, const double* __restrict__ R,
                                                         double* __restrict__ Y) {
  __shared__ double D[TRB][TRB + 1];
  for (int u = threadIdx.x; u < nb * nb; u += 256) {
    const int i = u / nb, j = u % nb;
    D[i][j] = R[(long long)(r0 + i) * l + r0 + j];
  }
  __syncthreads();
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= l) return;
  double y[TRB];
#pragma unroll
  for (int r = 0; r < TRB; ++r) y[r] = (r < nb) ? Y[(long long)(r0 + r) * l + c] : 0.0;
#pragma unroll
  for (int r = TRB - 1; r >= 0; --r) {
    if (r < nb) {
      double v = y[r];
#pragma unroll
      for (int k = r + 1; k < TRB; ++k)
        if (k < nb) v -= D[r][k] * y[k];
      y[r] = v / D[r][r];
    }
  }
#pragma unroll
  for (int r = 0; r < TRB; ++r)
    if (r < nb) Y[(long long)(r0 + r) * l + c] = y[r];
}

}  // namespace

hipError_t trtri_upper(int l, const double* R, double* Y, hipStream_t st) {
  const int last = ((l - 1) / TRB) * TRB;
  for (int r0 = last; r0 >= 0; r0 -= TRB) {
    const int nb = (l - r0 < TRB) ? (l - r0) : TRB;
    hipLaunchKernelGGL(eye_rows_kernel, dim3((unsigned)(((long long)nb * l + 255) / 256)), dim3(256), 0, st, l, r0, nb, Y);
    KOT_HIP_TRY(hipGetLastError());
    const int below = l - r0 - nb;
    if (below > 0) {
      GemmArgs g{};
      g.transa = 0; g.transb = 0; g.m = nb; g.n = l; g.k = below; g.alpha = -1.0; g.beta = 1.0;
      g.A = R + (long long)r0 * l + r0 + nb; g.lda = l;
      g.B = Y + (long long)(r0 + nb) * l; g.ldb = l;
      g.C = Y + (long long)r0 * l; g.ldc = l; g.batch = 1;
      KOT_HIP_TRY(gemm_f64(g, st));
    }
    hipLaunchKernelGGL(trsv_block_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, r0, nb, R, Y);
    KOT_HIP_TRY(hipGetLastError());
  }
  return hipSuccess;
}

hipError_t gram_build(int l, int d, const double* xf, const double* yf, double sigma, double* Q, double* K,
                      hipStream_t st) {
  dim3 grid((l + 15) / 16, (l + 15) / 16);
  hipLaunchKernelGGL(gram_kernel, grid, dim3(256), 0, st, l, d, xf, yf, 1.0 / (2.0 * sigma * sigma), Q, K);
  return hipGetLastError();
}

hipError_t mean_embedding(int n, int l, int d, const double* samples, const double* pts, double sigma, double* w,
                          hipStream_t st) {
  if (d > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(embed_kernel, dim3((l + EPT - 1) / EPT), dim3(256), 0, st, n, l, d, samples, pts,
                     1.0 / (2.0 * sigma * sigma), w);
  return hipGetLastError();
}

hipError_t mean_gram(int n, int d, const double* x, double sigma, double* out, double* part, hipStream_t st) {
  if (d > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(gram_rowsum_kernel, dim3(n), dim3(256), 0, st, n, d, x, 1.0 / (2.0 * sigma * sigma), part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(sum_scale_kernel, dim3(1), dim3(256), 0, st, n, part, 1.0 / ((double)n * (double)n), out);
  return hipGetLastError();
}

hipError_t build_z(int l, int d, const double* xf, const double* yf, const double* wmu, const double* wnu, double lam2,
                   double* z, double* wsum, hipStream_t st) {
  hipLaunchKernelGGL(z_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, d, xf, yf, wmu, wnu, lam2, z, wsum);
  return hipGetLastError();
}

hipError_t cholesky_upper(int l, const double* A, double eps, double* R, double* W, int* info, hipStream_t st) {
  const long long nn = (long long)l * l;
  const int eb = (int)((nn + 255) / 256);
  KOT_HIP_TRY(hipMemsetAsync(info, 0, sizeof(int), st));
  hipLaunchKernelGGL(copy_jitter_kernel, dim3(eb), dim3(256), 0, st, l, A, eps, W);
  KOT_HIP_TRY(hipGetLastError());
  for (int k0 = 0; k0 < l; k0 += CB) {
    const int nb = (l - k0 < CB) ? (l - k0) : CB;
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, st, l, k0, nb, W, info);
    KOT_HIP_TRY(hipGetLastError());
    const int rest = l - k0 - nb;
    if (rest <= 0) break;
    hipLaunchKernelGGL(trsm_panel_kernel, dim3((rest + 63) / 64), dim3(256), 0, st, l, k0, nb, W);
    KOT_HIP_TRY(hipGetLastError());
    // W22 -= L21 L21^T  (full trailing block; keeps it symmetric)
    GemmArgs g{};
    g.transa = 0; g.transb = 1; g.m = rest; g.n = rest; g.k = nb;
    g.alpha = -1.0; g.beta = 1.0;
    g.A = W + (long long)(k0 + nb) * l + k0; g.lda = l;
    g.B = W + (long long)(k0 + nb) * l + k0; g.ldb = l;
    g.C = W + (long long)(k0 + nb) * l + (k0 + nb); g.ldc = l;
    g.batch = 1;
    KOT_HIP_TRY(gemm_f64(g, st));
  }
  hipLaunchKernelGGL(lower_to_upper_kernel, dim3(eb), dim3(256), 0, st, l, W, R);
  return hipGetLastError();
}

}  // namespace kot
