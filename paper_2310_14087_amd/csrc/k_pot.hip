// Kantorovich potentials and transport map from the dual solution (Section 3): the maximizers of Eq. (3.2),
//   u(x) = (w_mu(x) - sum_i gamma_i k_X(x~_i, x)) / (2 lambda2),   w_mu(x) = (1/n) sum_j k_X(x_j, x),
// and T(x) = x - grad u(x) for the cost |x - y|^2 / 2, with grad_x k(a, x) = k(a, x) (a - x) / sigma^2.
// One pass over the "sources" (the n samples with weight 1/n, then the l filling points with weight -gamma_i)
// accumulates, per query point, s0 = sum_j w_j k_j and g = sum_j w_j k_j (a_j - x).  FP64 vector ALU.
#include "kot_internal.h"
#include <algorithm>

namespace kot {
namespace {

// Query block of 256 (one query per thread) x source split blockIdx.y; sources staged in LDS in chunks of CH.
// D >= d is the padded dimension (zero coordinates beyond d add nothing).  part[(split * m + i) * (D + 1)]
// holds (s0, g_0 .. g_{D-1}).
template <int D>
__global__ __launch_bounds__(256) void pot_part_kernel(int m, int d, const double* __restrict__ q,
                                                       const double* __restrict__ samples, int ns,
                                                       const double* __restrict__ fill, int l,
                                                       const double* __restrict__ gamma, double inv2s2, int per,
                                                       double* __restrict__ part) {
  constexpr int CH = D <= 16 ? 256 : 64;
  __shared__ double src[CH][D];
  __shared__ double wt[CH];
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int total = ns + l;
  const int s0 = blockIdx.y * per, s1 = min(total, s0 + per);
  double x[D], g[D];
#pragma unroll
  for (int k = 0; k < D; ++k) {
    x[k] = (i < m && k < d) ? q[(long long)i * d + k] : 0.0;
    g[k] = 0.0;
  }
  double acc = 0.0;
  for (int c0 = s0; c0 < s1; c0 += CH) {
    const int cn = min(CH, s1 - c0);
    __syncthreads();
    {
      // every load of a thread in flight together (register buffer), then staged
      constexpr int PER = CH * D / 256;
      double v[PER];
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int u = threadIdx.x + 256 * e, j = u / D, k = u - j * D;
        const int sidx = c0 + j;
        v[e] = 0.0;
        if (j < cn && k < d) v[e] = (sidx < ns) ? samples[(long long)sidx * d + k] : fill[(long long)(sidx - ns) * d + k];
      }
#pragma unroll
      for (int e = 0; e < PER; ++e) {
        const int u = threadIdx.x + 256 * e;
        src[u / D][u % D] = v[e];
      }
    }
    for (int j = threadIdx.x; j < CH; j += 256) {
      const int sidx = c0 + j;
      wt[j] = (j < cn) ? ((sidx < ns) ? 1.0 / ns : -gamma[sidx - ns]) : 0.0;
    }
    __syncthreads();
    for (int j = 0; j < cn; ++j) {
      double d2 = 0.0;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const double a = src[j][k] - x[k];
        d2 += a * a;
      }
      const double w = wt[j] * exp(-d2 * inv2s2);
      acc += w;
#pragma unroll
      for (int k = 0; k < D; ++k) g[k] += w * (src[j][k] - x[k]);
    }
  }
  if (i < m) {
    double* out = part + ((long long)blockIdx.y * m + i) * (D + 1);
    out[0] = acc;
#pragma unroll
    for (int k = 0; k < D; ++k) out[1 + k] = g[k];
  }
}

// Sum of the splits in order; u = s0 / (2 lambda2); T = x - g / (sigma^2 2 lambda2).
__global__ void pot_final_kernel(int m, int d, int D, int splits, const double* __restrict__ part,
                                 const double* __restrict__ q, double inv_2l2, double inv_s2, double* __restrict__ u,
                                 double* __restrict__ T) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const long long stride = (long long)m * (D + 1);
  const double* p = part + (long long)i * (D + 1);
  double s = 0.0;
  for (int sp = 0; sp < splits; ++sp) s += p[sp * stride];
  u[i] = s * inv_2l2;
  if (T) {
    for (int k = 0; k < d; ++k) {
      double gk = 0.0;
      for (int sp = 0; sp < splits; ++sp) gk += p[sp * stride + 1 + k];
      T[(long long)i * d + k] = q[(long long)i * d + k] - gk * inv_s2 * inv_2l2;
    }
  }
}

}  // namespace

int potential_dim(int d) {
  int D = 4;
  while (D < d) D *= 2;
  return D;
}

size_t potential_part_size(int m, int d, int splits) {
  return (size_t)splits * m * (potential_dim(d) + 1);
}

int potential_splits(int m, int ns, int l) {
  const int qb = (m + 255) / 256;
  int s = std::max(1, 1024 / qb);
  s = std::min(s, std::max(1, (ns + l) / 256));
  return s;
}

hipError_t potential_eval(int m, int d, const double* q, const double* samples, int ns, const double* fill, int l,
                          const double* gamma, double sigma, double lam2, int splits, double* part, double* u,
                          double* T, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  if (d < 1 || d > 64 || splits < 1) return hipErrorInvalidValue;
  const int D = potential_dim(d);
  const int total = ns + l;
  const int per = (total + splits - 1) / splits;
  dim3 grid((m + 255) / 256, splits);
  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);
  Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
  // per (query, source) pair: 3d flops for the distance, the exponential, 3d + 2 for the weighted sums
  if (pf) pf->begin(st, PROF_POTENTIAL, (double)m * total * (6.0 * d + 3.0), 8.0 * ((double)m * (2 * d + 1) + (double)total * d));
#define KOT_POT(DD) \
  if (D == DD) hipLaunchKernelGGL(pot_part_kernel<DD>, grid, dim3(256), 0, st, m, d, q, samples, ns, fill, l, gamma, inv2s2, per, part);
  KOT_POT(4) KOT_POT(8) KOT_POT(16) KOT_POT(32) KOT_POT(64)
#undef KOT_POT
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(pot_final_kernel, dim3((m + 255) / 256), dim3(256), 0, st, m, d, D, splits, part, q,
                     1.0 / (2.0 * lam2), 1.0 / (sigma * sigma), u, T);
  if (pf) pf->end(st);
  return hipGetLastError();
}

}  // namespace kot
