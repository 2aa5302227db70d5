// Reduced-precision GEMMs for the CG matvec chain (Algorithm 1): inputs FP32 in global memory, products on the
// matrix cores in FP32 (v_mfma_f32_16x16x4f32), BF16 (v_mfma_f32_16x16x16bf16_1k, operands rounded to
// bfloat16) or split BF16 (each operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi); the product is
// hi*hi + hi*lo + lo*hi, about 16 significant bits from three BF16 products), accumulation in FP32.  The
// first product of the chain carries the Hadamard weight Psi of Section 4.3 in its epilogue.
#include "kot_internal.h"
#include <algorithm>

namespace kot {

typedef float flt4 __attribute__((ext_vector_type(4)));
typedef short shrt4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int LBM = 64, LBN = 64, LBK = 32;
constexpr int LMK = LBK + 1;  // [row][k] tiles (lanes along k)
constexpr int LKM = LBN + 4;  // [k][col] tiles (lanes along col)

__device__ __forceinline__ short to_bf16(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float((unsigned)(unsigned short)h << 16); }
// hi and lo parts of four values
__device__ __forceinline__ void split4(const float f[4], shrt4& hi, shrt4& lo) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const short h = to_bf16(f[q]);
    hi[q] = h;
    lo[q] = to_bf16(f[q] - from_bf16(h));
  }
}

// Psi weight of entry (r, j) (eigen-index r, ascending eigenvalues w, alpha = [l-a, l)); see psi_kernel.
__device__ __forceinline__ double psi_weight(int r, int j, int l, int a, double mu, const double* __restrict__ w,
                                             int complement, double diag_scale, double off_scale) {
  const int split = l - a;
  const bool r_in = r >= split, j_in = j >= split;
  if (r_in == j_in) return diag_scale / mu;
  const int ia = r_in ? r : j, ib = r_in ? j : r;
  const double sa = w[ia], sb = -w[ib];
  const double one_m_eta = sb / (sa + sb), eta = sa / (sa + sb);
  return complement ? off_scale * (one_m_eta * (1.0 + mu) / (mu * (mu + one_m_eta)))
                    : off_scale * (eta / (mu + one_m_eta));
}

// C (m x n) = A (m x k, row-major, rows along k) diag(s) op(B); op(B) = B^T (TB: B is n x k) or B (k x n).
// blockIdx.z = K split: with splits > 1 the raw partial tile goes to part[split][m][n] and the reduction
// applies the epilogue.
// MODE: 0 FP32, 1 BF16, 2 split BF16
template <int MODE, bool TB, bool PSI>
__global__ __launch_bounds__(256) void gemm_lowp_kernel(LowpArgs g, int splits, int kchunk, float* __restrict__ part) {
  __shared__ float As[LBM * LMK];
  __shared__ float Bs[LBK * LKM > LBN * LMK ? LBK * LKM : LBN * LMK];
  const int M = g.m, N = g.n;
  const int kbeg = blockIdx.z * kchunk, K = min(g.k, kbeg + kchunk);
  const int m0 = blockIdx.y * LBM, n0 = blockIdx.x * LBN;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int r16 = lane & 15, k4 = lane >> 4;
  flt4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < K; k0 += LBK) {
    {  // A rows, lanes along k
      const int kk = t & 31, mm = t >> 5;
      const int gk = k0 + kk;
      const float sc = (g.s && gk < K) ? (float)g.s[gk] : 1.f;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gm = m0 + mm + 8 * u;
        As[(mm + 8 * u) * LMK + kk] = (gm < M && gk < K) ? g.A[(long long)gm * g.lda + gk] * sc : 0.f;
      }
    }
    if (TB) {  // B[n][k], lanes along k -> [n][k]
      const int kk = t & 31, nn = t >> 5;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gn = n0 + nn + 8 * u, gk = k0 + kk;
        Bs[(nn + 8 * u) * LMK + kk] = (gn < N && gk < K) ? g.B[(long long)gn * g.ldb + gk] : 0.f;
      }
    } else {   // B[k][n], lanes along n -> [k][n]
      const int nn = t & 63, kk = t >> 6;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int gn = n0 + nn, gk = k0 + kk + 4 * u;
        Bs[(kk + 4 * u) * LKM + nn] = (gn < N && gk < K) ? g.B[(long long)gk * g.ldb + gn] : 0.f;
      }
    }
    __syncthreads();
    if (MODE == 1) {
#pragma unroll
      for (int ks = 0; ks < LBK; ks += 16) {
        shrt4 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float* ap = As + (wm * 32 + i * 16 + r16) * LMK + ks + 4 * k4;
          a[i] = shrt4{to_bf16(ap[0]), to_bf16(ap[1]), to_bf16(ap[2]), to_bf16(ap[3])};
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn * 32 + j * 16 + r16, kb = ks + 4 * k4;
          if (TB) {
            const float* bp = Bs + col * LMK + kb;
            b[j] = shrt4{to_bf16(bp[0]), to_bf16(bp[1]), to_bf16(bp[2]), to_bf16(bp[3])};
          } else {
            b[j] = shrt4{to_bf16(Bs[kb * LKM + col]), to_bf16(Bs[(kb + 1) * LKM + col]),
                         to_bf16(Bs[(kb + 2) * LKM + col]), to_bf16(Bs[(kb + 3) * LKM + col])};
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    } else if (MODE == 2) {
#pragma unroll
      for (int ks = 0; ks < LBK; ks += 16) {
        shrt4 ah[2], al[2], bh[2], bl[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          const float* ap = As + (wm * 32 + i * 16 + r16) * LMK + ks + 4 * k4;
          const float f[4] = {ap[0], ap[1], ap[2], ap[3]};
          split4(f, ah[i], al[i]);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn * 32 + j * 16 + r16, kb = ks + 4 * k4;
          float f[4];
          if (TB) {
            const float* bp = Bs + col * LMK + kb;
            f[0] = bp[0]; f[1] = bp[1]; f[2] = bp[2]; f[3] = bp[3];
          } else {
            f[0] = Bs[kb * LKM + col]; f[1] = Bs[(kb + 1) * LKM + col];
            f[2] = Bs[(kb + 2) * LKM + col]; f[3] = Bs[(kb + 3) * LKM + col];
          }
          split4(f, bh[j], bl[j]);
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bl[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah[i], bh[j], acc[i][j], 0, 0, 0);
          }
      }
    } else {
#pragma unroll
      for (int ks = 0; ks < LBK; ks += 4) {
        float a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[(wm * 32 + i * 16 + r16) * LMK + ks + k4];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const int col = wn * 32 + j * 16 + r16, kk = ks + k4;
          b[j] = TB ? Bs[col * LMK + kk] : Bs[kk * LKM + col];
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // accumulator layout of both 16x16 f32-output instructions: lane L holds D[4*(L/16) + v][L%16]
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + i * 16 + 4 * k4 + v;
        const int col = n0 + wn * 32 + j * 16 + r16;
        if (row < M && col < N) {
          float r = acc[i][j][v];
          if (splits > 1) {
            part[((long long)blockIdx.z * M + row) * N + col] = r;
          } else {
            if (PSI) r *= (float)psi_weight(g.r0 + row, col, g.l, g.a, g.mu, g.w, g.complement, g.diag_scale, g.off_scale);
            g.C[(long long)row * g.ldc + col] = r;
          }
        }
      }
}

// C = sum over splits of the partial tiles (fixed order), then the Psi weight when requested.
__global__ void lowp_reduce_kernel(LowpArgs g, int splits, int psi, const float* __restrict__ part) {
  const long long mn = (long long)g.m * g.n;
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= mn) return;
  float r = 0.f;
  for (int q = 0; q < splits; ++q) r += part[q * mn + u];
  const int row = (int)(u / g.n), col = (int)(u % g.n);
  if (psi) r *= (float)psi_weight(g.r0 + row, col, g.l, g.a, g.mu, g.w, g.complement, g.diag_scale, g.off_scale);
  g.C[(long long)row * g.ldc + col] = r;
}

__global__ void f64_to_f32_kernel(long long n, const double* __restrict__ x, float* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// y[j] += alpha * sum_{r < m} A[r][j] * B[r][j]  (FP32 products, FP64 sums; 16 slabs then fixed order)
__global__ __launch_bounds__(256) void diag_dot_lowp_part(int m, int n, const float* __restrict__ A, int lda,
                                                          const float* __restrict__ B, int ldb, double* __restrict__ part) {
  const int col = blockIdx.x * 64 + (threadIdx.x & 63);
  const int sub = threadIdx.x >> 6;
  const int slab = blockIdx.y;
  const int per = (m + 15) / 16;
  const int s0 = slab * per, s1 = min(m, s0 + per);
  double acc = 0.0;
  if (col < n)
    for (int r = s0 + sub; r < s1; r += 4) acc += (double)(A[(long long)r * lda + col] * B[(long long)r * ldb + col]);
  __shared__ double red[4][64];
  red[sub][threadIdx.x & 63] = acc;
  __syncthreads();
  if (sub == 0 && col < n)
    part[(long long)slab * n + col] = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
}
__global__ void diag_dot_lowp_final(int n, double alpha, const double* __restrict__ part, double* __restrict__ y) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n) return;
  double s = 0.0;
  for (int p = 0; p < 16; ++p) s += part[(long long)p * n + col];
  y[col] += alpha * s;
}

}  // namespace

hipError_t gemm_lowp(const LowpArgs& g, int mode, bool psi, hipStream_t st) {
  if (g.m <= 0 || g.n <= 0 || g.k <= 0) return hipErrorInvalidValue;
  const int tiles = ((g.n + LBN - 1) / LBN) * ((g.m + LBM - 1) / LBM);
  // K split for thin products (the chain runs with m = min(|alpha|, l - |alpha|) rows): about one workgroup
  // per CU, at least 64 of K per split, partials in the split-K workspace (as floats)
  int splits = 1;
  if (tiles < 256 && g.k >= 128) splits = std::min(16, std::min((256 + tiles - 1) / tiles, g.k / 64));
  float* part = reinterpret_cast<float*>(g_gemm_ws);
  while (splits > 1 && (!part || (size_t)splits * g.m * g.n > 2 * g_gemm_ws_cap)) --splits;
  int kchunk = g.k;
  if (splits > 1) {
    kchunk = ((g.k + splits - 1) / splits + LBK - 1) / LBK * LBK;
    splits = (g.k + kchunk - 1) / kchunk;
  }
  dim3 grid((g.n + LBN - 1) / LBN, (g.m + LBM - 1) / LBM, splits);
  Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
  if (pf) pf->begin(st, mode ? PROF_GEMM_BF16 : PROF_GEMM_F32, 2.0 * g.m * g.n * (double)g.k,
                    4.0 * ((double)g.m * g.k + (double)g.k * g.n + (double)g.m * g.n));
#define KOT_LOWP(MD, TB_, PS) \
  if (mode == MD && (g.transb != 0) == TB_ && psi == PS) \
    hipLaunchKernelGGL((gemm_lowp_kernel<MD, TB_, PS>), grid, dim3(256), 0, st, g, splits, kchunk, part);
#define KOT_LOWP_MODE(MD) \
  KOT_LOWP(MD, true, true) KOT_LOWP(MD, true, false) KOT_LOWP(MD, false, true) KOT_LOWP(MD, false, false)
  KOT_LOWP_MODE(0) KOT_LOWP_MODE(1) KOT_LOWP_MODE(2)
#undef KOT_LOWP_MODE
#undef KOT_LOWP
  if (splits > 1) {
    const long long mn = (long long)g.m * g.n;
    hipLaunchKernelGGL(lowp_reduce_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, st, g, splits, psi ? 1 : 0,
                       (const float*)part);
  }
  if (pf) pf->end(st);
  return hipGetLastError();
}

hipError_t f64_to_f32(long long n, const double* x, float* y, hipStream_t st) {
  hipLaunchKernelGGL(f64_to_f32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, x, y);
  return hipGetLastError();
}

hipError_t diag_dot_lowp(int m, int n, double alpha, const float* A, int lda, const float* B, int ldb, double* y,
                         double* part, hipStream_t st) {
  if (n <= 0 || m <= 0) return hipSuccess;
  hipLaunchKernelGGL(diag_dot_lowp_part, dim3((n + 63) / 64, 16), dim3(256), 0, st, m, n, A, lda, B, ldb, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(diag_dot_lowp_final, dim3((n + 255) / 256), dim3(256), 0, st, n, alpha, part, y);
  return hipGetLastError();
}


// ==== BF16 chain on gfx950 (v_mfma_f32_16x16x32_bf16) ========================================================
// Per Newton direction the chain's operand B = P^T R is rounded once into bfloat16 copies, zero-padded to a
// leading dimension ldp (a multiple of 64): Bh = bf16(B) and BhT = bf16(B^T) (so that both products read their
// second operand along K), and for split BF16 the low parts Bl = bf16(B - Bh), BlT.  Per matvec two kernels
// run the chain:
//   chain 1: H = Psi o (B_set diag(v) B^T), written as bfloat16 (hi, and lo for split BF16), zero beyond col l;
//   chain 2: y_j += alpha sum_r D_rj (H B)_rj with D = B_set in FP32, the product never written: each workgroup
//            reduces its tile's column dots into part[tile row][j], a small kernel sums those in a fixed order.
// Both are NT products with K contiguous in memory: a lane's 8 consecutive bfloat16 of K (16 bytes) are one
// MFMA operand fragment, loaded straight from global memory (L2-resident operands) without LDS staging.
// Workgroup: 8 wavefronts on a 32 x 64 output tile, wavefront w taking K steps w, w + 8, ... (32 each); the
// partial tiles (or, for chain 2, their column dots) are summed through LDS in a fixed order.
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ unsigned short bf16_bits(float f) {  // round to nearest even
  unsigned u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_val(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct Frag { uint4 u; };
__device__ __forceinline__ bf16x8 as_bf16x8(const uint4& u) { return __builtin_bit_cast(bf16x8, u); }
__device__ __forceinline__ uint4 load_frag(const unsigned short* __restrict__ p, bool ok) {
  return ok ? *reinterpret_cast<const uint4*>(p) : make_uint4(0u, 0u, 0u, 0u);
}
__device__ __forceinline__ float frag_elem(const uint4& u, int q) {
  const unsigned w = (q < 2) ? u.x : (q < 4) ? u.y : (q < 6) ? u.z : u.w;
  return bf16_val((unsigned short)((q & 1) ? (w >> 16) : (w & 0xFFFFu)));
}
__device__ __forceinline__ uint4 pack_frag(const float x[8]) {
  uint4 u;
  u.x = bf16_bits(x[0]) | ((unsigned)bf16_bits(x[1]) << 16);
  u.y = bf16_bits(x[2]) | ((unsigned)bf16_bits(x[3]) << 16);
  u.z = bf16_bits(x[4]) | ((unsigned)bf16_bits(x[5]) << 16);
  u.w = bf16_bits(x[6]) | ((unsigned)bf16_bits(x[7]) << 16);
  return u;
}

// Psi weight in FP32 (the result is rounded to bfloat16): see psi_weight.
__device__ __forceinline__ float psi_weight_f(int r, int j, int l, int a, float mu, const double* __restrict__ w,
                                              int complement, float diag_scale, float off_scale) {
  const int split = l - a;
  const bool r_in = r >= split, j_in = j >= split;
  if (r_in == j_in) return diag_scale / mu;
  const int ia = r_in ? r : j, ib = r_in ? j : r;
  const float sa = (float)w[ia], sb = (float)(-w[ib]);
  const float inv = 1.0f / (sa + sb);
  const float one_m_eta = sb * inv, eta = sa * inv;
  return complement ? off_scale * (one_m_eta * (1.0f + mu) / (mu * (mu + one_m_eta)))
                    : off_scale * (eta / (mu + one_m_eta));
}

constexpr int CTM = 32, CTN = 64, CK = 32;

__global__ __launch_bounds__(256) void chain_prep_kernel(int l, int ldp, const double* __restrict__ B,
                                                         unsigned short* __restrict__ Bh, unsigned short* __restrict__ BhT,
                                                         unsigned short* __restrict__ Bl, unsigned short* __restrict__ BlT) {
  // 32 x 32 tile (row block y, col block x) through LDS for the transposed copies
  __shared__ float T[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    const float x = (r < l && c < l) ? (float)B[(long long)r * l + c] : 0.0f;
    const double xd = (r < l && c < l) ? B[(long long)r * l + c] : 0.0;
    const unsigned short h = bf16_bits(x);
    Bh[(long long)r * ldp + c] = h;
    if (Bl) Bl[(long long)r * ldp + c] = bf16_bits((float)(xd - (double)bf16_val(h)));
    T[ty + 8 * q][tx] = x;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + ty + 8 * q, r = r0 + tx;  // BhT[c][r] = B[r][c]
    const float x = T[tx][ty + 8 * q];
    const unsigned short h = bf16_bits(x);
    BhT[(long long)c * ldp + r] = h;
    if (BlT) {
      const double xd = (r < l && c < l) ? B[(long long)r * l + c] : 0.0;
      BlT[(long long)c * ldp + r] = bf16_bits((float)(xd - (double)bf16_val(h)));
    }
  }
}

// KIND 1: H = Psi o (A diag(v) B^T) with A = Bh rows r0.. (and Bl), B = Bh (and Bl); writes Hh (and Hl).
// KIND 2: part[y][j] = sum over the tile's rows of D[r][j] (H Bt^T)[r][j], A = Hh (and Hl), B = BhT (and BlT).
// CW wavefronts per workgroup share the K steps round-robin; each loads the fragments of its next K step
// before issuing the products of the current one.
constexpr int CW = 8;

struct ChainFrags {
  uint4 ah[2], al[2], bh[4], bl[4];
};

template <bool SPLIT, int KIND>
__device__ __forceinline__ void chain_load(const ChainArgs& g, const unsigned short* Ah, const unsigned short* Al,
                                           const unsigned short* Bh, const unsigned short* Bl, int m0, int n0,
                                           int r16, int k, ChainFrags& f) {
  const int ldp = g.ldp;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int row = m0 + 16 * i + r16;
    const bool ok = row < g.m;
    f.ah[i] = load_frag(Ah + (long long)row * ldp + k, ok);
    if (SPLIT) f.al[i] = load_frag(Al + (long long)row * ldp + k, ok);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = n0 + 16 * j + r16;
    f.bh[j] = load_frag(Bh + (long long)col * ldp + k, true);
    if (SPLIT) f.bl[j] = load_frag(Bl + (long long)col * ldp + k, true);
  }
}

template <bool SPLIT, int KIND>
__global__ __launch_bounds__(64 * CW) void chain_bf16_kernel(ChainArgs g) {
  __shared__ float red[KIND == 1 ? CW : 1][CTM][CTN + 1];
  __shared__ double colsum[KIND == 2 ? CW : 1][CTN];
  const int M = g.m, ldp = g.ldp;
  const int m0 = blockIdx.y * CTM, n0 = blockIdx.x * CTN;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r16 = lane & 15, kg = (lane >> 4) * 8;
  const unsigned short* Ah = KIND == 1 ? g.Bh + (long long)g.r0 * ldp : g.Hh;
  const unsigned short* Al = KIND == 1 ? (SPLIT ? g.Bl + (long long)g.r0 * ldp : nullptr) : g.Hl;
  const unsigned short* Bh = KIND == 1 ? g.Bh : g.BhT;
  const unsigned short* Bl = KIND == 1 ? g.Bl : g.BlT;
  flt4 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = flt4{0.f, 0.f, 0.f, 0.f};
  const int nsteps = ldp / CK;
  ChainFrags cur, nxt;
  if (wv < nsteps) chain_load<SPLIT, KIND>(g, Ah, Al, Bh, Bl, m0, n0, r16, wv * CK + kg, cur);
  for (int s = wv; s < nsteps; s += CW) {
    const int k = s * CK + kg;
    if (s + CW < nsteps) chain_load<SPLIT, KIND>(g, Ah, Al, Bh, Bl, m0, n0, r16, k + CW * CK, nxt);
    if (KIND == 1) {  // A <- A diag(v), rounded again
      float vk[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) vk[q] = (k + q < g.l) ? (float)g.v[k + q] : 0.f;
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        float x[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) x[q] = (frag_elem(cur.ah[i], q) + (SPLIT ? frag_elem(cur.al[i], q) : 0.f)) * vk[q];
        cur.ah[i] = pack_frag(x);
        if (SPLIT) {
          float y[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) y[q] = x[q] - frag_elem(cur.ah[i], q);
          cur.al[i] = pack_frag(y);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        if (SPLIT) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(cur.ah[i]), as_bf16x8(cur.bl[j]), acc[i][j], 0, 0, 0);
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(cur.al[i]), as_bf16x8(cur.bh[j]), acc[i][j], 0, 0, 0);
        }
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(cur.ah[i]), as_bf16x8(cur.bh[j]), acc[i][j], 0, 0, 0);
      }
    cur = nxt;
  }
  // accumulator lane L holds rows 4 (L/16) + v of column L % 16
  if (KIND == 1) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) red[wv][16 * i + 4 * (lane >> 4) + v][16 * j + r16] = acc[i][j][v];
    __syncthreads();
    // 2048 entries, 4 per thread: column t % 64, rows t / 64 + 8 q; the CW partials summed in a fixed order
    const int c = threadIdx.x & 63, rb = threadIdx.x >> 6;
    const int col = n0 + c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = rb + 8 * q, row = m0 + r;
      if (row >= M || col >= ldp) continue;
      float x = 0.f;
#pragma unroll
      for (int w2 = 0; w2 < CW; ++w2) x += red[w2][r][c];
      x = (col < g.l) ? x * psi_weight_f(g.r0 + row, col, g.l, g.a, (float)g.mu, g.w, g.complement,
                                         (float)g.diag_scale, (float)g.off_scale)
                      : 0.f;
      const unsigned short h = bf16_bits(x);
      g.Hh[(long long)row * ldp + col] = h;
      if (SPLIT) g.Hl[(long long)row * ldp + col] = bf16_bits(x - bf16_val(h));
    }
  } else {
    // column dots of this wavefront's partial tile: sum_r D[r][c] acc[r][c] over its 32 rows, then over the
    // lane groups holding other rows (fixed butterfly), then over the wavefronts in order
    double cs[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + 16 * j + r16;
      double t = 0.0;
      if (col < g.l) {
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int row = m0 + 16 * i + 4 * (lane >> 4) + v;
            if (row < M) t += (double)(g.D[(long long)row * g.ldd + col] * acc[i][j][v]);
          }
      }
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      cs[j] = t;
    }
    if (lane < 16) {
#pragma unroll
      for (int j = 0; j < 4; ++j) colsum[wv][16 * j + lane] = cs[j];
    }
    __syncthreads();
    if (threadIdx.x < CTN) {
      const int c = threadIdx.x, col = n0 + c;
      if (col < g.l) {
        double sum = 0.0;
#pragma unroll
        for (int w2 = 0; w2 < CW; ++w2) sum += colsum[w2][c];
        g.part[(long long)blockIdx.y * g.l + col] = sum;
      }
    }
  }
}

__global__ void chain_final_kernel(int n, int tiles, double alpha, const double* __restrict__ part, double* __restrict__ y) {
  const int col = blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= n) return;
  double s = 0.0;
  for (int t = 0; t < tiles; ++t) s += part[(long long)t * n + col];
  y[col] += alpha * s;
}

}  // namespace

int chain_ldp(int l) { return (l + 63) / 64 * 64; }

hipError_t chain_prep(int l, int ldp, const double* B, unsigned short* Bh, unsigned short* BhT, unsigned short* Bl,
                      unsigned short* BlT, hipStream_t st) {
  dim3 grid(ldp / 32, ldp / 32);
  hipLaunchKernelGGL(chain_prep_kernel, grid, dim3(256), 0, st, l, ldp, B, Bh, BhT, Bl, BlT);
  return hipGetLastError();
}

hipError_t chain_bf16(const ChainArgs& g, bool split, hipStream_t st) {
  if (g.m <= 0) return hipSuccess;
  const int tiles_m = (g.m + CTM - 1) / CTM;
  Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
  const double fl = 2.0 * g.m * (double)g.l * g.l * (split ? 3.0 : 1.0);
  const double by = 2.0 * ((double)g.m * g.l + (double)g.l * g.l) * (split ? 2.0 : 1.0) + 2.0 * g.m * (double)g.l;
  {
    dim3 grid(g.ldp / CTN, tiles_m);
    if (pf) pf->begin(st, PROF_GEMM_BF16, fl, by);
    if (split) hipLaunchKernelGGL((chain_bf16_kernel<true, 1>), grid, dim3(64 * CW), 0, st, g);
    else hipLaunchKernelGGL((chain_bf16_kernel<false, 1>), grid, dim3(64 * CW), 0, st, g);
    if (pf) pf->end(st);
    KOT_HIP_TRY(hipGetLastError());
  }
  {
    dim3 grid((g.l + CTN - 1) / CTN, tiles_m);
    if (pf) pf->begin(st, PROF_GEMM_BF16, fl, by);
    if (split) hipLaunchKernelGGL((chain_bf16_kernel<true, 2>), grid, dim3(64 * CW), 0, st, g);
    else hipLaunchKernelGGL((chain_bf16_kernel<false, 2>), grid, dim3(64 * CW), 0, st, g);
    KOT_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(chain_final_kernel, dim3((g.l + 255) / 256), dim3(256), 0, st, g.l, tiles_m, g.alpha, g.part, g.y);
    if (pf) pf->end(st);
  }
  return hipGetLastError();
}

}  // namespace kot
