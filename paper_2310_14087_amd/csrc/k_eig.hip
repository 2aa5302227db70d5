// Symmetric eigendecomposition Z = P diag(w) P^T (Eq. 4.4) by two-sided block Jacobi.
//
// Indices are cut into blocks of 8; a sweep is a round-robin tournament over the blocks (circle method), so
// every pair of blocks meets once per sweep.  In one round the pairs are disjoint:
//   1. pair_solve: one wavefront per pair loads its 16x16 subproblem into LDS and diagonalizes it with
//      cyclic scalar Jacobi (8 disjoint rotations at a time), giving an orthogonal 16x16 U;
//   2. apply_A / apply_V: A <- G^T A G and V <- V G with G the block-diagonal of the U's, each 16x16 tile
//      updated by two 16x16x16 products on the matrix cores (v_mfma_f64_16x16x4f64; accumulator lane L
//      holds rows L/16 + 4v, v = 0..3, of column L%16).
// Sweeps repeat until off(A) <= tol * |A|_F; the eigenvalues are diag(A), sorted ascending with V's
// columns permuted alongside.  A warm start replaces (Z, I) by (P0^T Z P0, P0).
#include "kot_internal.h"
#include <vector>
#include <cmath>

namespace kot {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BSZ = 8;    // block width
constexpr int SLOT = 16;  // indices per pair

__device__ __forceinline__ int pair_slot_index(int p, int q, int s, int l) {
  const int g = (s < BSZ) ? p * BSZ + s : q * BSZ + (s - BSZ);
  return (g < l) ? g : -1;
}

// 16-player circle ordering: in sub-round r, pair 0 = (15, r), pair k = ((r+k)%15, (r-k+15)%15).
__device__ __forceinline__ void circle16(int r, int k, int& a, int& b) {
  if (k == 0) { a = 15; b = r; }
  else { a = (r + k) % 15; b = (r - k + 15) % 15; }
}

__global__ __launch_bounds__(64) void pair_solve_kernel(int l, const double* __restrict__ A, const int2* __restrict__ pairs,
                                                        double* __restrict__ Uout, int* __restrict__ flag,
                                                        const double* __restrict__ thresh_ptr, int max_inner) {
  const double thresh = *thresh_ptr;
  __shared__ double S[SLOT][SLOT + 1];
  __shared__ double U[SLOT][SLOT + 1];
  __shared__ double cs[8][2];
  __shared__ int idx[SLOT];
  __shared__ int any_rot;
  const int k = blockIdx.x;
  const int2 pq = pairs[k];
  const int lane = threadIdx.x;
  if (lane < SLOT) idx[lane] = pair_slot_index(pq.x, pq.y, lane, l);
  if (lane == 0) any_rot = 0;
  __syncthreads();
  for (int u = lane; u < SLOT * SLOT; u += 64) {
    const int i = u >> 4, j = u & 15;
    const int gi = idx[i], gj = idx[j];
    S[i][j] = (gi >= 0 && gj >= 0) ? A[(long long)gi * l + gj] : 0.0;
    U[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    // largest off-diagonal magnitude of the subproblem
    double mx = 0.0;
    for (int u = lane; u < SLOT * SLOT; u += 64) {
      const int i = u >> 4, j = u & 15;
      if (i != j) mx = fmax(mx, fabs(S[i][j]));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
    if (mx <= thresh) break;
    for (int r = 0; r < 15; ++r) {
      if (lane < 8) {
        int a, b;
        circle16(r, lane, a, b);
        if (a > b) { const int t = a; a = b; b = t; }
        const double apq = S[a][b];
        double c = 1.0, s = 0.0;
        if (fabs(apq) > thresh) {
          const double theta = (S[b][b] - S[a][a]) / (2.0 * apq);
          const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
          c = 1.0 / sqrt(t * t + 1.0);
          s = t * c;
          any_rot = 1;
        }
        cs[lane][0] = c;
        cs[lane][1] = s;
      }
      __syncthreads();
      // columns: S <- S J, U <- U J   (16 rows x 8 pairs, 2 tasks per lane)
      for (int u = lane; u < 128; u += 64) {
        const int row = u >> 3, pk = u & 7;
        int a, b;
        circle16(r, pk, a, b);
        if (a > b) { const int t = a; a = b; b = t; }
        const double c = cs[pk][0], s = cs[pk][1];
        if (s != 0.0) {
          const double x = S[row][a], y = S[row][b];
          S[row][a] = c * x - s * y;
          S[row][b] = s * x + c * y;
          const double ux = U[row][a], uy = U[row][b];
          U[row][a] = c * ux - s * uy;
          U[row][b] = s * ux + c * uy;
        }
      }
      __syncthreads();
      // rows: S <- J^T S
      for (int u = lane; u < 128; u += 64) {
        const int col = u >> 3, pk = u & 7;
        int a, b;
        circle16(r, pk, a, b);
        if (a > b) { const int t = a; a = b; b = t; }
        const double c = cs[pk][0], s = cs[pk][1];
        if (s != 0.0) {
          const double x = S[a][col], y = S[b][col];
          S[a][col] = c * x - s * y;
          S[b][col] = s * x + c * y;
        }
      }
      __syncthreads();
      if (lane < 8) {
        int a, b;
        circle16(r, lane, a, b);
        if (cs[lane][1] != 0.0) { S[a][b] = 0.0; S[b][a] = 0.0; }
      }
      __syncthreads();
    }
  }
  double* Uk = Uout + (long long)k * SLOT * SLOT;
  for (int u = lane; u < SLOT * SLOT; u += 64) Uk[u] = U[u >> 4][u & 15];
  if (lane == 0) flag[k] = any_rot;
}

// A_PQ <- U_P^T A_PQ U_Q for every pair-block tile (P, Q).
__global__ __launch_bounds__(64) void apply_A_kernel(int l, double* __restrict__ A, const int2* __restrict__ pairs,
                                                     const double* __restrict__ Ub, const int* __restrict__ flag) {
  const int P = blockIdx.y, Qb = blockIdx.x;
  if (!flag[P] && !flag[Qb]) return;
  __shared__ double M[SLOT][SLOT + 1];
  __shared__ double T[SLOT][SLOT + 1];
  __shared__ int ip[SLOT], iq[SLOT];
  const int lane = threadIdx.x;
  const int2 pp = pairs[P], qq = pairs[Qb];
  if (lane < SLOT) {
    ip[lane] = pair_slot_index(pp.x, pp.y, lane, l);
    iq[lane] = pair_slot_index(qq.x, qq.y, lane, l);
  }
  __syncthreads();
  for (int u = lane; u < SLOT * SLOT; u += 64) {
    const int i = u >> 4, j = u & 15;
    const int gi = ip[i], gj = iq[j];
    M[i][j] = (gi >= 0 && gj >= 0) ? A[(long long)gi * l + gj] : 0.0;
  }
  __syncthreads();
  const double* UP = Ub + (long long)P * SLOT * SLOT;
  const double* UQ = Ub + (long long)Qb * SLOT * SLOT;
  const int r16 = lane & 15, k4 = lane >> 4;
  dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < SLOT; ks += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[r16][ks + k4], UQ[(ks + k4) * SLOT + r16], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) T[k4 + 4 * v][r16] = acc[v];
  __syncthreads();
  dbl4 acc2 = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < SLOT; ks += 4)
    acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(UP[(ks + k4) * SLOT + r16], T[ks + k4][r16], acc2, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int gi = ip[k4 + 4 * v], gj = iq[r16];
    if (gi >= 0 && gj >= 0) A[(long long)gi * l + gj] = acc2[v];
  }
}

// V[R, idx_P] <- V[R, idx_P] U_P for 16-row slabs R.
__global__ __launch_bounds__(64) void apply_V_kernel(int l, double* __restrict__ V, const int2* __restrict__ pairs,
                                                     const double* __restrict__ Ub, const int* __restrict__ flag) {
  const int P = blockIdx.y;
  if (!flag[P]) return;
  const int r0 = blockIdx.x * SLOT;
  __shared__ double M[SLOT][SLOT + 1];
  __shared__ int ip[SLOT];
  const int lane = threadIdx.x;
  const int2 pp = pairs[P];
  if (lane < SLOT) ip[lane] = pair_slot_index(pp.x, pp.y, lane, l);
  __syncthreads();
  for (int u = lane; u < SLOT * SLOT; u += 64) {
    const int i = u >> 4, j = u & 15;
    const int gj = ip[j];
    M[i][j] = (r0 + i < l && gj >= 0) ? V[(long long)(r0 + i) * l + gj] : 0.0;
  }
  __syncthreads();
  const double* UP = Ub + (long long)P * SLOT * SLOT;
  const int r16 = lane & 15, k4 = lane >> 4;
  dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < SLOT; ks += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[r16][ks + k4], UP[(ks + k4) * SLOT + r16], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + k4 + 4 * v, gj = ip[r16];
    if (row < l && gj >= 0) V[(long long)row * l + gj] = acc[v];
  }
}

// part[b] = (sum of off-diagonal squares, sum of all squares) over a grid-stride slice; fixed order.
__global__ __launch_bounds__(256) void offnorm_part_kernel(int l, const double* __restrict__ A, double* __restrict__ part) {
  __shared__ double r0[256], r1[256];
  const long long nn = (long long)l * l;
  double off = 0.0, all = 0.0;
  for (long long u = (long long)blockIdx.x * 256 + threadIdx.x; u < nn; u += (long long)gridDim.x * 256) {
    const double v = A[u];
    const int i = (int)(u / l), j = (int)(u % l);
    all += v * v;
    if (i != j) off += v * v;
  }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { r0[threadIdx.x] += r0[threadIdx.x + h]; r1[threadIdx.x] += r1[threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = r0[0]; part[2 * blockIdx.x + 1] = r1[0]; }
}

__global__ __launch_bounds__(256) void offnorm_final_kernel(int nb, const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double r0[256], r1[256];
  double off = 0.0, all = 0.0;
  for (int b = threadIdx.x; b < nb; b += 256) { off += part[2 * b]; all += part[2 * b + 1]; }
  r0[threadIdx.x] = off;
  r1[threadIdx.x] = all;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { r0[threadIdx.x] += r0[threadIdx.x + h]; r1[threadIdx.x] += r1[threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { out[0] = sqrt(r0[0]); out[1] = sqrt(r1[0]); }
}

__global__ void eye_kernel(int l, double* __restrict__ V) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  V[u] = ((u / l) == (u % l)) ? 1.0 : 0.0;
}

// Single-workgroup bitonic sort of (diag(A), index) ascending; writes w and perm.
__global__ __launch_bounds__(1024) void sort_diag_kernel(int l, int npow2, const double* __restrict__ A, double* __restrict__ w,
                                                         int* __restrict__ perm) {
  extern __shared__ unsigned char smem[];
  double* key = reinterpret_cast<double*>(smem);
  int* val = reinterpret_cast<int*>(key + npow2);
  for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
    key[i] = (i < l) ? A[(long long)i * l + i] : INFINITY;
    val[i] = i;
  }
  __syncthreads();
  for (int size = 2; size <= npow2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int i = threadIdx.x; i < npow2; i += blockDim.x) {
        const int j = i ^ stride;
        if (j > i) {
          const bool up = ((i & size) == 0);
          const double ki = key[i], kj = key[j];
          const int vi = val[i], vj = val[j];
          const bool gt = (ki > kj) || (ki == kj && vi > vj);
          if (gt == up) { key[i] = kj; key[j] = ki; val[i] = vj; val[j] = vi; }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < l; i += blockDim.x) { w[i] = key[i]; perm[i] = val[i]; }
}

__global__ void permute_cols_kernel(int l, const double* __restrict__ V, const int* __restrict__ perm, double* __restrict__ P) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  P[u] = V[(long long)i * l + perm[j]];
}

}  // namespace

struct EigWork {
  int lmax = 0;
  // one captured sweep (all rounds) per (l, A/V buffers); replayed with hipGraphLaunch
  int graph_l = -1;
  const double* graph_tmp = nullptr;
  hipGraphExec_t graph = nullptr;
  bool graph_failed = false;
  int nb = -1;                // block count of the current pair table
  int2* pairs = nullptr;      // device [(nb-1) * nb/2]
  double* U = nullptr;        // device [npairs_max * 256]
  int* flag = nullptr;        // device [npairs_max]
  double* part = nullptr;     // device [2 * 512]
  double* norms = nullptr;    // device [4]: off, |A|_F, rotation threshold
  double* hnorms = nullptr;   // pinned host [4]
  int* perm = nullptr;        // device [lmax]
};

EigWork* eig_work_create(int lmax) {
  EigWork* w = new EigWork();
  w->lmax = lmax;
  const int nbmax = ((lmax + BSZ - 1) / BSZ + 1) & ~1;
  const int npm = nbmax / 2;
  bool ok = hipMalloc(&w->pairs, sizeof(int2) * (size_t)(nbmax) * npm + 16) == hipSuccess &&
            hipMalloc(&w->U, sizeof(double) * (size_t)npm * 256) == hipSuccess &&
            hipMalloc(&w->flag, sizeof(int) * (size_t)npm) == hipSuccess &&
            hipMalloc(&w->part, sizeof(double) * 1024) == hipSuccess &&
            hipMalloc(&w->norms, sizeof(double) * 4) == hipSuccess &&
            hipHostMalloc(&w->hnorms, sizeof(double) * 4) == hipSuccess &&
            hipMalloc(&w->perm, sizeof(int) * (size_t)lmax) == hipSuccess;
  if (!ok) { eig_work_destroy(w); return nullptr; }
  return w;
}

void eig_work_destroy(EigWork* w) {
  if (!w) return;
  if (w->graph) hipGraphExecDestroy(w->graph);
  hipFree(w->pairs); hipFree(w->U); hipFree(w->flag); hipFree(w->part); hipFree(w->norms);
  hipHostFree(w->hnorms); hipFree(w->perm);
  delete w;
}

static hipError_t ensure_pairs(EigWork* w, int nb, hipStream_t st) {
  if (w->nb == nb) return hipSuccess;
  const int np = nb / 2;
  std::vector<int2> h((size_t)(nb - 1) * np);
  for (int r = 0; r < nb - 1; ++r) {
    for (int k = 0; k < np; ++k) {
      int a, b;
      if (k == 0) { a = nb - 1; b = r; }
      else { a = (r + k) % (nb - 1); b = (r - k + (nb - 1)) % (nb - 1); }
      h[(size_t)r * np + k] = make_int2(a, b);
    }
  }
  KOT_HIP_TRY(hipMemcpyAsync(w->pairs, h.data(), sizeof(int2) * h.size(), hipMemcpyHostToDevice, st));
  KOT_HIP_TRY(hipStreamSynchronize(st));
  w->nb = nb;
  return hipSuccess;
}

static hipError_t off_norm(EigWork* w, int l, const double* A, hipStream_t st, double* off, double* all) {
  const long long nn = (long long)l * l;
  int nbk = (int)((nn + 255) / 256);
  if (nbk > 512) nbk = 512;
  hipLaunchKernelGGL(offnorm_part_kernel, dim3(nbk), dim3(256), 0, st, l, A, w->part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(offnorm_final_kernel, dim3(1), dim3(256), 0, st, nbk, w->part, w->norms);
  KOT_HIP_TRY(hipGetLastError());
  KOT_HIP_TRY(hipMemcpyAsync(w->hnorms, w->norms, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  KOT_HIP_TRY(hipStreamSynchronize(st));
  *off = w->hnorms[0];
  *all = w->hnorms[1];
  return hipSuccess;
}

hipError_t eigh_jacobi(EigWork* w, int l, const double* Z, const double* P0, double* P, double* wv, double* tmp,
                       int max_sweeps, double tol, int* sweeps, double* rel_off, hipStream_t st) {
  if (l > w->lmax) return hipErrorInvalidValue;
  double* A = tmp;
  double* V = tmp + (long long)l * l;
  const long long nn = (long long)l * l;
  const int eb = (int)((nn + 255) / 256);
  if (P0) {
    // A = P0^T Z P0 (Z P0 staged in V; P0 may alias the output P), then V = P0
    GemmArgs g{};
    g.transa = 0; g.transb = 0; g.m = l; g.n = l; g.k = l; g.alpha = 1.0; g.beta = 0.0;
    g.A = Z; g.lda = l; g.B = P0; g.ldb = l; g.C = V; g.ldc = l; g.batch = 1;
    KOT_HIP_TRY(gemm_f64(g, st));
    g.transa = 1; g.A = P0; g.B = V; g.C = A;
    KOT_HIP_TRY(gemm_f64(g, st));
    KOT_HIP_TRY(symmetrize(l, A, st));
    KOT_HIP_TRY(hipMemcpyAsync(V, P0, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
  } else {
    KOT_HIP_TRY(hipMemcpyAsync(A, Z, sizeof(double) * nn, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(eye_kernel, dim3(eb), dim3(256), 0, st, l, V);
    KOT_HIP_TRY(hipGetLastError());
  }
  int nb = (l + BSZ - 1) / BSZ;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  KOT_HIP_TRY(ensure_pairs(w, nb, st));
  const int np = nb / 2;
  double off = 0.0, all = 0.0;
  KOT_HIP_TRY(off_norm(w, l, A, st, &off, &all));
  int s = 0;
  const double thresh_rel = 1e-18;
  auto launch_sweep = [&](hipStream_t s_) -> hipError_t {
    for (int r = 0; r < nb - 1; ++r) {
      const int2* pr = w->pairs + (size_t)r * np;
      hipLaunchKernelGGL(pair_solve_kernel, dim3(np), dim3(64), 0, s_, l, A, pr, w->U, w->flag, w->norms + 2, 8);
      KOT_HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(apply_A_kernel, dim3(np, np), dim3(64), 0, s_, l, A, pr, w->U, w->flag);
      KOT_HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL(apply_V_kernel, dim3((l + SLOT - 1) / SLOT, np), dim3(64), 0, s_, l, V, pr, w->U, w->flag);
      KOT_HIP_TRY(hipGetLastError());
    }
    return hipSuccess;
  };
  // flops of one sweep: per round 2 x 2 x 16^3 per A tile and 2 x 16^3 per V tile
  const double sweep_flops = (double)(nb - 1) * (4.0 * 4096.0 * np * np + 2.0 * 4096.0 * ((l + SLOT - 1) / SLOT) * np);
  while (off > tol * all && s < max_sweeps) {
    w->hnorms[2] = thresh_rel * all;
    KOT_HIP_TRY(hipMemcpyAsync(w->norms + 2, w->hnorms + 2, sizeof(double), hipMemcpyHostToDevice, st));
    if (!w->graph_failed && (w->graph == nullptr || w->graph_l != l || w->graph_tmp != tmp)) {
      if (w->graph) { hipGraphExecDestroy(w->graph); w->graph = nullptr; }
      hipGraph_t gr = nullptr;
      bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
      if (ok) {
        const hipError_t le = launch_sweep(st);
        ok = hipStreamEndCapture(st, &gr) == hipSuccess && le == hipSuccess && gr != nullptr;
      }
      if (ok) ok = hipGraphInstantiate(&w->graph, gr, nullptr, nullptr, 0) == hipSuccess;
      if (gr) hipGraphDestroy(gr);
      if (!ok) {
        (void)hipGetLastError();
        w->graph = nullptr;
        w->graph_failed = true;
      } else {
        w->graph_l = l;
        w->graph_tmp = tmp;
      }
    }
    Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
    if (pf) pf->begin(st, PROF_EIG_ROUND, sweep_flops, 32.0 * l * (double)l * (nb - 1));
    if (w->graph) KOT_HIP_TRY(hipGraphLaunch(w->graph, st));
    else KOT_HIP_TRY(launch_sweep(st));
    if (pf) pf->end(st);
    ++s;
    KOT_HIP_TRY(off_norm(w, l, A, st, &off, &all));
  }
  *sweeps = s;
  *rel_off = (all > 0.0) ? off / all : 0.0;
  int npow2 = 1;
  while (npow2 < l) npow2 <<= 1;
  const size_t sm = (size_t)npow2 * (sizeof(double) + sizeof(int));
  if (sm > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sort_diag_kernel, dim3(1), dim3(1024), sm, st, l, npow2, A, wv, w->perm);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(permute_cols_kernel, dim3(eb), dim3(256), 0, st, l, V, w->perm, P);
  return hipGetLastError();
}

}  // namespace kot
