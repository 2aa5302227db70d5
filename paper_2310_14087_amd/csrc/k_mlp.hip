// Warm-start network kernels (FP32): a 3-layer perceptron applied row-wise to per-filling-point features,
// its MSE loss, backpropagation and Adam, plus the feature kernel and the weights used to lift a predicted
// dual into a multiplier X0.  GEMMs run on the matrix cores (v_mfma_f32_16x16x4f32).
#include "kot_internal.h"
#include <cmath>

namespace kot {

typedef float flt4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int FBM = 64, FBN = 64, FBK = 32;
constexpr int FKM = FBM + 4;   // k-major tile stride
constexpr int FMK = FBK + 1;   // m-major tile stride
constexpr int FTILE = FBK * FKM > FBM * FMK ? FBK * FKM : FBM * FMK;

// C = op(A) op(B) (+ beta C) (+ bias[col]) then relu (act == 1) or times (mask > 0) (mask != null).
// MFMA layout (16x16x4 f32): lane L supplies A[L%16][L/16], B[L/16][L%16]; accumulator lane L holds
// D[4*(L/16) + v][L%16].
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void gemm_f32_kernel(GemmF32Args g) {
  __shared__ float As[FTILE];
  __shared__ float Bs[FTILE];
  const int M = g.m, N = g.n, K = g.k;
  const int m0 = blockIdx.y * FBM, n0 = blockIdx.x * FBN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int r16 = lane & 15, k4 = lane >> 4;
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  // the next K slice is loaded into registers while the current one feeds the matrix cores
  float ra[8], rb[8];
  auto load = [&](int k0) {
    if (!TA) {  // A[m][k], lanes along k
      const int kk = t & 31, mm = t >> 5;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gm = m0 + mm + 8 * u, gk = k0 + kk;
        ra[u] = (gm < M && gk < K) ? g.A[(long long)gm * g.lda + gk] : 0.f;
      }
    } else {    // A[k][m], lanes along m
      const int mm = t & 63, kk = t >> 6;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gm = m0 + mm, gk = k0 + kk + 4 * u;
        ra[u] = (gm < M && gk < K) ? g.A[(long long)gk * g.lda + gm] : 0.f;
      }
    }
    if (!TB) {  // B[k][n], lanes along n
      const int nn = t & 63, kk = t >> 6;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gn = n0 + nn, gk = k0 + kk + 4 * u;
        rb[u] = (gn < N && gk < K) ? g.B[(long long)gk * g.ldb + gn] : 0.f;
      }
    } else {    // B[n][k], lanes along k
      const int kk = t & 31, nn = t >> 5;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gn = n0 + nn + 8 * u, gk = k0 + kk;
        rb[u] = (gn < N && gk < K) ? g.B[(long long)gn * g.ldb + gk] : 0.f;
      }
    }
  };
  auto store = [&]() {
    if (!TA) {
      const int kk = t & 31, mm = t >> 5;
#pragma unroll
      for (int u = 0; u < 8; ++u) As[(mm + 8 * u) * FMK + kk] = ra[u];
    } else {
      const int mm = t & 63, kk = t >> 6;
#pragma unroll
      for (int u = 0; u < 8; ++u) As[(kk + 4 * u) * FKM + mm] = ra[u];
    }
    if (!TB) {
      const int nn = t & 63, kk = t >> 6;
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[(kk + 4 * u) * FKM + nn] = rb[u];
    } else {
      const int kk = t & 31, nn = t >> 5;
#pragma unroll
      for (int u = 0; u < 8; ++u) Bs[(nn + 8 * u) * FMK + kk] = rb[u];
    }
  };
  load(0);
  store();
  __syncthreads();
  for (int k0 = 0; k0 < K; k0 += FBK) {
    const bool more = k0 + FBK < K;
    if (more) load(k0 + FBK);
#pragma unroll
    for (int ks = 0; ks < FBK; ks += 4) {
      float a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int m = wm * 32 + i * 16 + r16, k = ks + k4;
        a[i] = TA ? As[k * FKM + m] : As[m * FMK + k];
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int n = wn * 32 + j * 16 + r16, k = ks + k4;
        b[j] = TB ? Bs[n * FMK + k] : Bs[k * FKM + n];
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (more) {
      __syncthreads();
      store();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * k4 + v;
        const int col = n0 + wn * 32 + j * 16 + r16;
        if (row < M && col < N) {
          float* p = g.C + (long long)row * g.ldc + col;
          float r = acc[i][j][v];
          if (g.beta != 0.f) r += g.beta * (*p);
          if (g.bias) r += g.bias[col];
          if (g.act == 1) r = fmaxf(r, 0.f);
          if (g.mask) r = (g.mask[(long long)row * g.ldm + col] > 0.f) ? r : 0.f;
          *p = r;
        }
      }
}

// n == 1 with op(A) = A and op(B) = B (k x 1): one wavefront per row, the same epilogue as the GEMM.
__global__ __launch_bounds__(256) void gemv_f32_kernel(GemmF32Args g) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= g.m) return;
  const float* a = g.A + (long long)row * g.lda;
  float acc = 0.f;
  for (int c = lane; c < g.k; c += 64) acc += a[c] * g.B[(long long)c * g.ldb];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if (lane == 0) {
    float* p = g.C + (long long)row * g.ldc;
    float r = acc;
    if (g.beta != 0.f) r += g.beta * (*p);
    if (g.bias) r += g.bias[0];
    if (g.act == 1) r = fmaxf(r, 0.f);
    if (g.mask) r = (g.mask[(long long)row * g.ldm] > 0.f) ? r : 0.f;
    *p = r;
  }
}

// out[j] = sum_i X[i][j] over rows, in 16 fixed slabs then a fixed-order sum.
__global__ __launch_bounds__(256) void colsum_part_kernel(int rows, int cols, const float* __restrict__ X,
                                                          float* __restrict__ part) {
  const int col = blockIdx.x * 256 + threadIdx.x;
  const int slab = blockIdx.y;
  const int per = (rows + 15) / 16;
  const int r0 = slab * per, r1 = min(rows, r0 + per);
  if (col >= cols) return;
  float s = 0.f;
  for (int r = r0; r < r1; ++r) s += X[(long long)r * cols + col];
  part[(long long)slab * cols + col] = s;
}
__global__ void colsum_final_kernel(int cols, const float* __restrict__ part, float* __restrict__ out) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= cols) return;
  float s = 0.f;
  for (int q = 0; q < 16; ++q) s += part[(long long)q * cols + col];
  out[col] = s;
}

// r = out - y; dout = 2 r / N; part[b] = partial sum of r^2 (double)
__global__ __launch_bounds__(256) void mse_kernel(int n, const float* __restrict__ out, const float* __restrict__ y,
                                                  float* __restrict__ dout, double* __restrict__ part) {
  __shared__ double red[256];
  double acc = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const float r = out[i] - y[i];
    dout[i] = 2.f * r / (float)n;
    acc += (double)r * (double)r;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ __launch_bounds__(256) void mse_final_kernel(int nb, int n, const double* __restrict__ part, double* __restrict__ loss) {
  __shared__ double red[256];
  red[threadIdx.x] = threadIdx.x < nb ? part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (double)n;
}

__global__ void adam_kernel(int n, float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Per-point features, bounded and free of the problem's scale (so a network trained at one size applies at
// another): with f0 = z_i/(lambda1 Q_ii)
//   0 max(f0, -2)        1 max(f0, -1)           2 (Q 1)_i/Q_ii - 1     3 (K 1)_i/K_ii - 1
//   4 ((K o K) 1)_i/K_ii^2 - 1                   5 Q_ii - 2             6 K_ii - 1
//   7 min(wsum_i/|z_i|, 10)                      8 fraction of points with f0 < -1 (pooled)
//   9 mean of max(f0, -1) (pooled)               10 0 (reserved)        11 1
__global__ void feature_kernel(int l, const double* __restrict__ Q, const double* __restrict__ z, const double* __restrict__ wsum,
                               const double* __restrict__ K, const double* __restrict__ rs, double lam1,
                               const double* __restrict__ pooled, float* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double qii = Q[(long long)i * l + i];
  const double kii = K[(long long)i * l + i];
  const double f0 = z[i] / (lam1 * qii);
  const double az = fabs(z[i]);
  const double f[kFeatures] = {fmax(f0, -2.0), fmax(f0, -1.0), rs[i] / qii - 1.0, rs[l + i] / kii - 1.0,
                               rs[2 * l + i] / (kii * kii) - 1.0, qii - 2.0, kii - 1.0,
                               az > 0.0 ? fmin(wsum[i] / az, 10.0) : 10.0, pooled[0], pooled[1], 0.0, 1.0};
  for (int c = 0; c < kFeatures; ++c) X[(long long)i * kFeatures + c] = (float)f[c];
}
// pooled[0] = fraction of points with f0 < -1, pooled[1] = mean of max(f0, -1)
__global__ __launch_bounds__(256) void pooled_kernel(int l, const double* __restrict__ Q, const double* __restrict__ z,
                                                     double lam1, double* __restrict__ pooled) {
  __shared__ double r0[256], r1[256];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < l; i += 256) {
    const double f0 = z[i] / (lam1 * Q[(long long)i * l + i]);
    a += (f0 < -1.0) ? 1.0 : 0.0;
    b += fmax(f0, -1.0);
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { r0[threadIdx.x] += r0[threadIdx.x + h]; r1[threadIdx.x] += r1[threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { pooled[0] = r0[0] / l; pooled[1] = r1[0] / l; }
}
__global__ __launch_bounds__(256) void rowsum3_kernel(int l, const double* __restrict__ A, const double* __restrict__ B,
                                                      const double* __restrict__ C, double* __restrict__ rs) {
  __shared__ double red[3][256];
  const int i = blockIdx.x;
  double a = 0.0, b = 0.0, c = 0.0;
  for (int j = threadIdx.x; j < l; j += 256) {
    a += A[(long long)i * l + j];
    b += B[(long long)i * l + j];
    c += C[(long long)i * l + j];
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  red[2][threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) {
      red[0][threadIdx.x] += red[0][threadIdx.x + h];
      red[1][threadIdx.x] += red[1][threadIdx.x + h];
      red[2][threadIdx.x] += red[2][threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) { rs[i] = red[0][0]; rs[l + i] = red[1][0]; rs[2 * l + i] = red[2][0]; }
}

__global__ void f32_to_f64_scaled_kernel(int n, const float* __restrict__ x, double s, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = s * (double)x[i];
}

// d[i] = ((Q g)_i - z_i) / (2 lam2) where the constraint is predicted active (g_i <= -0.9 lambda1) and that
// value is positive, else 0; part[b] accumulates (sum d, count d > 0) per block.
__global__ __launch_bounds__(256) void lift_diag_kernel(int l, const double* __restrict__ Qg, const double* __restrict__ z,
                                                        const double* __restrict__ g, double lam1, double lam2,
                                                        double* __restrict__ d, double* __restrict__ part) {
  __shared__ double rs[256], rc[256];
  double s = 0.0, c = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < l; i += gridDim.x * 256) {
    const double y = (Qg[i] - z[i]) / (2.0 * lam2);
    const double v = (g[i] <= -0.9 * lam1 && y > 0.0) ? y : 0.0;
    d[i] = v;
    s += v;
    c += (v > 0.0) ? 1.0 : 0.0;
  }
  rs[threadIdx.x] = s;
  rc[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { rs[threadIdx.x] += rs[threadIdx.x + h]; rc[threadIdx.x] += rc[threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = rs[0]; part[2 * blockIdx.x + 1] = rc[0]; }
}
// thr = frac * (sum d / count d>0); d[i] = 0 where d[i] < thr
__global__ __launch_bounds__(256) void lift_threshold_kernel(int l, int nb, const double* __restrict__ part, double frac,
                                                             double* __restrict__ d) {
  __shared__ double thr;
  if (threadIdx.x == 0) {
    double s = 0.0, c = 0.0;
    for (int b = 0; b < nb; ++b) { s += part[2 * b]; c += part[2 * b + 1]; }
    thr = (c > 0.0) ? frac * s / c : 0.0;
  }
  __syncthreads();
  for (int i = blockIdx.x * 256 + threadIdx.x; i < l; i += gridDim.x * 256)
    if (d[i] < thr) d[i] = 0.0;
}

__global__ void closed_start_kernel(int l, const double* __restrict__ Q, const double* __restrict__ z, double lam1,
                                    double* __restrict__ g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < l) g[i] = fmax(z[i] / Q[(long long)i * l + i], -lam1);
}

}  // namespace

// gamma0_i = max(z_i / Q_ii, -lambda1): the minimizer of Eq. (3.4) when Q is diagonal and R orthogonal (the LMI
// is then the box gamma >= -lambda1), i.e. lambda1 times the network's first input feature, clipped.
hipError_t closed_start(int l, const double* Q, const double* z, double lam1, double* g, hipStream_t st) {
  hipLaunchKernelGGL(closed_start_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, Q, z, lam1, g);
  return hipGetLastError();
}


hipError_t gemm_f32(const GemmF32Args& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0 || g.k <= 0) return hipErrorInvalidValue;
  if (g.n == 1 && g.ta == 0 && g.tb == 0) {
    hipLaunchKernelGGL(gemv_f32_kernel, dim3((g.m + 3) / 4), dim3(256), 0, st, g);
    return hipGetLastError();
  }
  dim3 grid((g.n + FBN - 1) / FBN, (g.m + FBM - 1) / FBM);
  if (g.ta == 0 && g.tb == 0) hipLaunchKernelGGL((gemm_f32_kernel<false, false>), grid, dim3(256), 0, st, g);
  else if (g.ta == 0 && g.tb == 1) hipLaunchKernelGGL((gemm_f32_kernel<false, true>), grid, dim3(256), 0, st, g);
  else if (g.ta == 1 && g.tb == 0) hipLaunchKernelGGL((gemm_f32_kernel<true, false>), grid, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((gemm_f32_kernel<true, true>), grid, dim3(256), 0, st, g);
  return hipGetLastError();
}

hipError_t colsum_f32(int rows, int cols, const float* X, float* out, float* part, hipStream_t st) {
  hipLaunchKernelGGL(colsum_part_kernel, dim3((cols + 255) / 256, 16), dim3(256), 0, st, rows, cols, X, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(colsum_final_kernel, dim3((cols + 255) / 256), dim3(256), 0, st, cols, part, out);
  return hipGetLastError();
}

hipError_t mse_grad(int n, const float* out, const float* y, float* dout, double* loss, double* part, hipStream_t st) {
  int nb = (n + 255) / 256;
  if (nb > 256) nb = 256;
  hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, st, n, out, y, dout, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(mse_final_kernel, dim3(1), dim3(256), 0, st, nb, n, part, loss);
  return hipGetLastError();
}

hipError_t adam_f32(int n, float* th, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int t,
                    hipStream_t st) {
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  hipLaunchKernelGGL(adam_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, th, g, m, v, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

hipError_t features(int l, const double* Q, const double* z, const double* wsum, const double* K, const double* KK,
                    double lam1, double* rs, double* pooled, float* X, hipStream_t st) {
  hipLaunchKernelGGL(rowsum3_kernel, dim3(l), dim3(256), 0, st, l, Q, K, KK, rs);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(pooled_kernel, dim3(1), dim3(256), 0, st, l, Q, z, lam1, pooled);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(feature_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, Q, z, wsum, K, rs, lam1, pooled, X);
  return hipGetLastError();
}

hipError_t f32_to_f64_scaled(int n, const float* x, double s, double* y, hipStream_t st) {
  hipLaunchKernelGGL(f32_to_f64_scaled_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, x, s, y);
  return hipGetLastError();
}

hipError_t lift_diag(int l, const double* Qg, const double* z, const double* g, double lam1, double lam2, double frac,
                     double* d, double* part, hipStream_t st) {
  int nb = (l + 255) / 256;
  if (nb > 64) nb = 64;
  hipLaunchKernelGGL(lift_diag_kernel, dim3(nb), dim3(256), 0, st, l, Qg, z, g, lam1, lam2, d, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(lift_threshold_kernel, dim3(nb), dim3(256), 0, st, l, nb, part, frac, d);
  return hipGetLastError();
}

}  // namespace kot
