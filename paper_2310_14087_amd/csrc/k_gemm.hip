// FP64 GEMM on CDNA4 matrix cores (v_mfma_f64_16x16x4f64) with LDS-staged 64x64x16 tiles, and the
// column-dot reduction used for Phi(X)_i = R[:,i]^T (X R)[:,i] and the diagonal extract of the CG matvec.
#include "kot_internal.h"

namespace kot {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int PAD = 4;  // row pad (doubles) of the LDS tiles

// One 64x64 output tile per workgroup of 256 threads = 4 waves in a 2x2 grid; each wave owns 32x32 =
// 2x2 MFMA blocks of 16x16.  MFMA operand layout (16x16x4 f64): lane L supplies A[L%16][L/16] and
// B[L/16][L%16]; the accumulator lane L holds D[L/16 + 4*v][L%16], v = 0..3.
template <bool TA, bool TB, bool SC>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[BK][BM + PAD];
  __shared__ double Bs[BK][BN + PAD];
  const int bz = blockIdx.z;
  const double* __restrict__ A = g.A + bz * g.sA;
  const double* __restrict__ B = g.B + bz * g.sB;
  const double* __restrict__ S = SC ? g.s + bz * g.sS : nullptr;
  double* __restrict__ C = g.C + bz * g.sC;
  const int M = g.m, N = g.n, K = g.k;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  dbl4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  for (int k0 = 0; k0 < K; k0 += BK) {
    // ---- stage op(A)[m0:m0+64, k0:k0+16] into As[k][m] ----
    if (!TA) {  // A[m*lda + k]: 4 consecutive k per thread
      const int mm = t >> 2, kq = (t & 3) * 4;
      const int gm = m0 + mm;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gk = k0 + kq + u;
        double v = (gm < M && gk < K) ? A[(long long)gm * g.lda + gk] : 0.0;
        if (SC) v *= (gk < K) ? S[gk] : 0.0;
        As[kq + u][mm] = v;
      }
    } else {    // A[k*lda + m]: 4 consecutive m per thread
      const int kk = t >> 4, mq = (t & 15) * 4;
      const int gk = k0 + kk;
      const double sc = (SC && gk < K) ? S[gk] : 1.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gm = m0 + mq + u;
        double v = (gm < M && gk < K) ? A[(long long)gk * g.lda + gm] : 0.0;
        As[kk][mq + u] = SC ? v * sc : v;
      }
    }
    // ---- stage op(B)[k0:k0+16, n0:n0+64] into Bs[k][n] ----
    if (!TB) {  // B[k*ldb + n]
      const int kk = t >> 4, nq = (t & 15) * 4;
      const int gk = k0 + kk;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gn = n0 + nq + u;
        Bs[kk][nq + u] = (gn < N && gk < K) ? B[(long long)gk * g.ldb + gn] : 0.0;
      }
    } else {    // B[n*ldb + k]
      const int nn = t >> 2, kq = (t & 3) * 4;
      const int gn = n0 + nn;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int gk = k0 + kq + u;
        Bs[kq + u][nn] = (gn < N && gk < K) ? B[(long long)gn * g.ldb + gk] : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = As[ks + (lane >> 4)][wm * 32 + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = Bs[ks + (lane >> 4)][wn * 32 + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // ---- epilogue ----
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * v;
        const int col = n0 + wn * 32 + j * 16 + (lane & 15);
        if (row < M && col < N) {
          double* p = C + (long long)row * g.ldc + col;
          const double r = g.alpha * acc[i][j][v];
          *p = (g.beta == 0.0) ? r : r + g.beta * (*p);
        }
      }
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

hipEvent_t Profiler::get() {
  if (next == pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  return pool[next++];
}
void Profiler::begin(hipStream_t st, int cls, double flops, double bytes) {
  Rec r{cls, flops, bytes, get(), get()};
  if (r.a) hipEventRecord(r.a, st);
  recs.push_back(r);
}
void Profiler::end(hipStream_t st) {
  if (!recs.empty() && recs.back().b) hipEventRecord(recs.back().b, st);
}
void Profiler::clear() { recs.clear(); next = 0; }
Profiler::~Profiler() { for (auto e : pool) hipEventDestroy(e); }

hipError_t gemm_f64(const GemmArgs& g, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0 || g.batch <= 0) return hipSuccess;
  if (g.k <= 0) {  // C = beta C
    // handled by a k=1 launch with alpha = 0 would read A; do it explicitly instead
    return hipErrorInvalidValue;
  }
  dim3 grid((g.n + BN - 1) / BN, (g.m + BM - 1) / BM, g.batch);
  dim3 block(256);
  const bool sc = g.s != nullptr;
  Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
  // algorithmic work of the product: 2mnk flops; bytes = each operand and C read/written once
  if (pf) pf->begin(st, PROF_GEMM_F64, 2.0 * g.m * g.n * (double)g.k * g.batch,
                    8.0 * g.batch * ((double)g.m * g.k + (double)g.k * g.n + (g.beta != 0.0 ? 2.0 : 1.0) * g.m * g.n));
#define KOT_GEMM_CASE(TA, TB, SC_) \
  if (g.transa == TA && g.transb == TB && sc == SC_) { hipLaunchKernelGGL((gemm_f64_kernel<TA, TB, SC_>), grid, block, 0, st, g); if (pf) pf->end(st); return hipGetLastError(); }
  KOT_GEMM_CASE(0, 0, false) KOT_GEMM_CASE(0, 1, false) KOT_GEMM_CASE(1, 0, false) KOT_GEMM_CASE(1, 1, false)
  KOT_GEMM_CASE(0, 0, true) KOT_GEMM_CASE(0, 1, true) KOT_GEMM_CASE(1, 0, true) KOT_GEMM_CASE(1, 1, true)
#undef KOT_GEMM_CASE
  return hipErrorInvalidValue;
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
