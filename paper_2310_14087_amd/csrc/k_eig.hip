// Symmetric eigendecomposition Z = P diag(w) P^T (Eq. 4.4) by two-sided block Jacobi.
//
// Indices are cut into blocks of 8; a sweep is a round-robin tournament over the blocks (circle method), so
// every pair of blocks meets once per sweep.  In one round the pairs are disjoint:
//   1. pair_solve: one wavefront per pair loads its 16x16 subproblem into LDS and diagonalizes it with
//      cyclic scalar Jacobi (8 disjoint rotations at a time), giving an orthogonal 16x16 U;
//   2. apply (one launch): A <- G^T A G and V <- V G with G the block-diagonal of the U's, each 16x16 tile
//      updated by two 16x16x16 products on the matrix cores (v_mfma_f64_16x16x4f64; accumulator lane L
//      holds rows L/16 + 4v, v = 0..3, of column L%16).
// Sweeps repeat until off(A) <= tol * |A|_F, measured from the norms of the 8x8 blocks.  When few block
// pairs carry off-diagonal mass above a threshold (tau, chosen so that all pairs below it already satisfy the
// stopping test), a sweep rotates only those: they are packed into rounds of disjoint pairs, completed to a
// partition of the blocks by pairs that rotate nothing; otherwise the sweep is the full tournament, captured
// once per size as a HIP graph.  The eigenvalues are diag(A), sorted ascending (by ranks) with V's columns
// permuted alongside.  A warm start replaces (Z, I) by (P0^T Z P0, P0).
#include "kot_internal.h"
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

namespace kot {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int BSZ = 8;    // block width
constexpr int SLOT = 16;  // indices per pair

__device__ __forceinline__ int pair_slot_index(int p, int q, int s, int l) {
  const int g = (s < BSZ) ? p * BSZ + s : q * BSZ + (s - BSZ);
  return (g < l) ? g : -1;
}

// Index of slot s (0..15) of block pair (x, y) in the block-padded range (slots past l included).
__device__ __forceinline__ int slot_index(int2 pq, int s) { return (s < BSZ) ? pq.x * BSZ + s : pq.y * BSZ + (s - BSZ); }

// Blocked storage of the working matrices A and V during the sweeps: the 8x8 block (bi, bj) of the L x L matrix
// (L = 8 nb) occupies 64 consecutive doubles at (bi nb + bj) 64, row-major inside, so that a 16x16 tile of a
// block pair is four 512-byte runs.  Of the symmetric A only the lower blocks are kept (sym); V is kept
// transposed (V^T in the same storage).  Entries past l are zero and
// stay zero: no rotation involves an index past l (its entries of A are zero), so the U of every pair is the
// identity on such slots.
__host__ __device__ __forceinline__ long long blk(int nb, int i, int j) {
  return ((long long)(i >> 3) * nb + (j >> 3)) * 64 + (i & 7) * 8 + (j & 7);
}
// A is symmetric and only its lower blocks (bi >= bj) are kept: entry (i, j) lives at (i, j) or at (j, i).
__device__ __forceinline__ long long sym(int nb, int i, int j) {
  return ((i >> 3) >= (j >> 3)) ? blk(nb, i, j) : blk(nb, j, i);
}

// Round-robin tournament over nb (even) blocks, circle method: in round r < nb - 1, pair 0 = (nb-1, r) and
// pair k = ((r + k) mod (nb-1), (r - k) mod (nb-1)); every pair of blocks meets once in nb - 1 rounds.
__device__ __forceinline__ int2 round_pair(int r, int k, int nb) {
  const int m = nb - 1;
  if (k == 0) return make_int2(m, r);
  int a = r + k, b = r - k;
  if (a >= m) a -= m;
  if (b < 0) b += m;
  return make_int2(a, b);
}

// Pair k of a round: from the tournament formula, or from an explicit list (threshold sweeps).
__device__ __forceinline__ int2 get_pair(int round, int nb, const int2* __restrict__ list, int k) {
  return list ? list[k] : round_pair(round, k, nb);
}

// Index pair (a < b) that lane k (0..7) rotates in sub-round r of one visit of a block pair (slots 0-7: block
// p, 8-15: block q).  With `within`, sub-rounds 0-6 rotate the pairs inside each block (circle method on 8 indices:
// lanes 0-3 block p, lanes 4-7 block q) and sub-rounds 7-14 the cross pairs; otherwise the 8 sub-rounds rotate the
// cross pairs only: sub-round r pairs slot k with slot 8 + (k + r) mod 8.  A tournament sweep visits each block
// pair once and runs `within` in its first round only (where every block appears once), so every index pair is
// rotated exactly once per sweep: a cyclic Jacobi sweep in a parallel ordering.
__device__ __forceinline__ void pair_of_subround(int r, int k, int within, int& a, int& b) {
  if (within && r < 7) {
    const int kk = k & 3, off = (k < 4) ? 0 : 8;
    int x, y;
    if (kk == 0) { x = 7; y = r; }
    else { x = (r + kk) % 7; y = (r - kk + 7) % 7; }
    a = off + (x < y ? x : y);
    b = off + (x < y ? y : x);
  } else {
    const int rc = within ? r - 7 : r;
    a = k;
    b = 8 + (k + rc) % 8;
  }
}

// With an explicit list, pairs k >= kact only complete the partition of the blocks: they rotate nothing.
// One wavefront per pair runs cyclic Jacobi on the 16x16 subproblem S (8 disjoint rotations per sub-round,
// jacobi16): every lane applies S <- J^T S J to one 2x2 block (rows of pair lane/8, columns of pair lane%8; the
// blocks are disjoint, so the two-sided update is one read and one write of each entry) and U <- U J to two
// row segments.  The annihilated entries of the diagonal blocks are set to zero exactly.  Inner sweeps stop
// after a sweep that rotated nothing, or after max_inner sweeps.
// V <- V G of the previous round, in the same launch (it does not feed this round's pair solves): workgroups
// from npb on take four (pair, 16-row slab) items each, with the previous round's rotations.
struct VPrev {
  int active;          // 0 at a sweep's first round
  int round;           // previous round (tournament), or its explicit pair list below
  const int2* list;
  const double* U;
  const int* flag;
  double* V;
  int nslab;
};

__device__ __forceinline__ void v_slab_update(int l, int nb, const VPrev& vp, int item, int np,
                                              double (*M)[SLOT + 1], int* ip);

// Cyclic Jacobi on the 16x16 subproblem S staged in LDS (one wavefront; U starts as the identity).  Returns
// whether any rotation was applied.
__device__ __forceinline__ bool jacobi16(double (*S)[SLOT + 1], double (*U)[SLOT + 1], double2* cs, double thresh,
                                         int max_inner, int within);

__global__ __launch_bounds__(64) void pair_solve_kernel(int l, const double* __restrict__ A, int round, int nb,
                                                        const int2* __restrict__ list, int kact, int npb,
                                                        double* __restrict__ Uout, int* __restrict__ flag,
                                                        const double* __restrict__ thresh_ptr, int max_inner,
                                                        int within, VPrev vp, int np) {
  __shared__ double S[SLOT][SLOT + 1];
  __shared__ double U[SLOT][SLOT + 1];
  __shared__ double2 cs[8];
  __shared__ int idx[SLOT];
  if ((int)blockIdx.x >= npb) {
    const int base = ((int)blockIdx.x - npb) * 4;
#pragma unroll 1
    for (int q = 0; q < 4; ++q) v_slab_update(l, nb, vp, base + q, np, S, idx);
    return;
  }
  if (list && (int)blockIdx.x >= kact) {
    if (threadIdx.x == 0) flag[blockIdx.x] = 0;
    return;
  }
  const double thresh = *thresh_ptr;
  const int k = blockIdx.x;
  const int2 pq = get_pair(round, nb, list, k);
  const int lane = threadIdx.x;
  if (lane < SLOT) idx[lane] = pair_slot_index(pq.x, pq.y, lane, l);
  __syncthreads();
  // the four loads of a lane are issued together (register buffer), then staged
  double sv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = lane + 64 * q, i = u >> 4, j = u & 15;
    const int gi = idx[i], gj = idx[j];
    sv[q] = (gi >= 0 && gj >= 0) ? A[sym(nb, gi, gj)] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = lane + 64 * q, i = u >> 4, j = u & 15;
    S[i][j] = sv[q];
    U[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  const bool rotated_any = jacobi16(S, U, cs, thresh, max_inner, within);
  __syncthreads();
  double* Uk = Uout + (long long)k * SLOT * SLOT;
  for (int u = lane; u < SLOT * SLOT; u += 64) Uk[u] = U[u >> 4][u & 15];
  if (lane == 0) flag[k] = rotated_any ? 1 : 0;
}

// 1/sqrt(x) and 1/x for positive normal x: the hardware estimate refined by one third-order step,
// y0 (1 + e/2 + 3 e^2/8) with e = 1 - x y0^2, and y0 (1 + e + e^2) with e = 1 - x y0.
__device__ __forceinline__ double rsqrt_refined(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y0, y0, 1.0);
  return fma(y0 * e, fma(0.375, e, 0.5), y0);
}
__device__ __forceinline__ double rcp_refined(double x) {
  const double y0 = __builtin_amdgcn_rcp(x);
  const double e = fma(-x, y0, 1.0);
  return fma(y0, fma(e, e, e), y0);
}
// 1/sqrt(x) to within about half an ulp: a Newton step from rsqrt_refined with the residual 1 - x y^2 formed
// from the exact split of y^2 (y y = hi + lo), so its rounding errors carry no bias (a biased c would make the
// columns of V drift in norm over thousands of rotations).
__device__ __forceinline__ double rsqrt_accurate(double x) {
  const double y = rsqrt_refined(x);
  const double hi = y * y;
  const double lo = fma(y, y, -hi);
  const double e = fma(-x, lo, fma(-x, hi, 1.0));
  return fma(0.5 * y, e, y);
}

// Rotation J = [[c, s], [-s, c]] that annihilates apq in the 2x2 [[app, apq], [apq, aqq]] (J^T S J), the identity
// when |apq| <= thresh: t = tan of the angle is the root of t^2 + 2 theta t - 1 = 0 (theta = d / (2 apq),
// d = aqq - app) of smaller magnitude, t = 2 apq sgn(d) / (|d| + sqrt(d^2 + 4 apq^2)), c = 1/sqrt(1 + t^2),
// s = t c.  The square root and the reciprocals come from refined hardware estimates (c to about half an ulp);
// when d^2 + 4 apq^2 leaves the normal range the same root is formed with IEEE division and square root from
// theta.  The threshold is applied by selection, so the common path has no branch.
__device__ __forceinline__ void jacobi_rot(double app, double aqq, double apq, double thresh, double& c, double& sn) {
  const bool act = fabs(apq) > thresh;
  const double d = aqq - app;
  const double h = fma(d, d, 4.0 * apq * apq);
  const bool normal = h > 1e-290 && h < 1e290;
  double t;
  if (normal || !act) {
    const double hh = normal ? h : 1.0;
    const double r = hh * rsqrt_refined(hh);
    t = (d >= 0.0 ? 2.0 * apq : -2.0 * apq) * rcp_refined(fabs(d) + r);
  } else {
    const double theta = d / (2.0 * apq);
    t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
  }
  const double cc = rsqrt_accurate(fma(t, t, 1.0));
  c = act ? cc : 1.0;
  sn = act ? t * cc : 0.0;
}

// One wavefront, no barriers.  Lane (k1, k2) = (lane / 8, lane % 8) forms the rotation J_k2 of sub-round pair k2
// (the eight lanes with the same k2 compute the same one from the same entries); the lanes with k1 == k2 publish
// theirs in cs, from which every lane takes J_k1.  The lane then applies S <- J^T S J to the 2x2 block (rows of
// pair k1, columns of pair k2) and U <- U J_k1 to rows 2 k2, 2 k2 + 1; an identity rotation leaves the entries
// exactly as they are, so the updates run unconditionally.  A sub-round issues its LDS reads of S and U before
// its writes; the LDS operations of one wavefront complete in issue order, so every read sees the previous
// sub-round's writes and none sees this one's, and the compiler barriers keep that order in the code.  Cross
// visits (no within-block rotations: every round of a sweep but its first) run an unrolled 8-sub-round loop
// whose pair indices are k and 8 + (k + r) mod 8.
__device__ __forceinline__ bool jacobi16(double (*S)[SLOT + 1], double (*U)[SLOT + 1], double2* cs, double thresh,
                                         int max_inner, int within) {
  const int lane = threadIdx.x;
  const int k1 = lane >> 3, k2 = lane & 7;
  const int ur = 2 * k2;
  bool rotated_any = false;
  auto subround = [&](int a1, int b1, int a2, int b2, bool& act) {
    const double p2 = S[a2][b2], d2a = S[a2][a2], d2b = S[b2][b2];
    const double xaa = S[a1][a2], xab = S[a1][b2], xba = S[b1][a2], xbb = S[b1][b2];
    const double u0a = U[ur][a1], u0b = U[ur][b1], u1a = U[ur + 1][a1], u1b = U[ur + 1][b1];
    asm volatile("" ::: "memory");
    double c2, s2;
    jacobi_rot(d2a, d2b, p2, thresh, c2, s2);
    act = act || fabs(p2) > thresh;
    if (k1 == k2) cs[k2] = make_double2(c2, s2);
    asm volatile("" ::: "memory");
    const double2 j1 = cs[k1];
    const double c1 = j1.x, s1 = j1.y;
    // rows: J1^T x, then columns: (J1^T x) J2
    const double yaa = c1 * xaa - s1 * xba, yab = c1 * xab - s1 * xbb;
    const double yba = s1 * xaa + c1 * xba, ybb = s1 * xab + c1 * xbb;
    const double zaa = c2 * yaa - s2 * yab, zbb = s2 * yba + c2 * ybb;
    const bool annihilate = k1 == k2 && s1 != 0.0;
    const double zab = annihilate ? 0.0 : s2 * yaa + c2 * yab;
    const double zba = annihilate ? 0.0 : c2 * yba - s2 * ybb;
    S[a1][a2] = zaa; S[a1][b2] = zab; S[b1][a2] = zba; S[b1][b2] = zbb;
    U[ur][a1] = c1 * u0a - s1 * u0b;
    U[ur][b1] = s1 * u0a + c1 * u0b;
    U[ur + 1][a1] = c1 * u1a - s1 * u1b;
    U[ur + 1][b1] = s1 * u1a + c1 * u1b;
    asm volatile("" ::: "memory");
  };
  for (int sweep = 0; sweep < max_inner; ++sweep) {
    bool act = false;
    if (!within) {
#pragma unroll
      for (int r = 0; r < 8; ++r) subround(k1, 8 + ((k1 + r) & 7), k2, 8 + ((k2 + r) & 7), act);
    } else {
      for (int r = 0; r < 15; ++r) {
        int a1, b1, a2, b2;
        pair_of_subround(r, k1, within, a1, b1);
        pair_of_subround(r, k2, within, a2, b2);
        subround(a1, b1, a2, b2, act);
      }
    }
    if (!__any(act)) break;
    rotated_any = true;
  }
  return rotated_any;
}

// Item i = P * nslab + slab of the previous round: V[r0.., idx_P] <- V[r0.., idx_P] U_P on a 16-row slab (a
// pair without rotations is skipped).  The whole workgroup (one wavefront) takes the item; the barriers are
// uniform over it.
__device__ __forceinline__ void v_slab_update(int l, int nb, const VPrev& vp, int item, int np,
                                              double (*M)[SLOT + 1], int* ip) {
  if (!vp.active || item >= np * vp.nslab) return;
  const int P = item / vp.nslab, r0 = (item % vp.nslab) * SLOT;
  if (!vp.flag[P]) return;
  const int lane = threadIdx.x;
  const int2 pp = get_pair(vp.round, nb, vp.list, P);
  __syncthreads();  // the previous item's reads of M and ip are done
  if (lane < SLOT) ip[lane] = pair_slot_index(pp.x, pp.y, lane, l);
  __syncthreads();
  double mv[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = lane + 64 * q, i = u >> 4, j = u & 15;
    const int gj = ip[j];
    mv[q] = (r0 + i < l && gj >= 0) ? vp.V[blk(nb, gj, r0 + i)] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = lane + 64 * q;
    M[u >> 4][u & 15] = mv[q];
  }
  __syncthreads();
  const double* UP = vp.U + (long long)P * SLOT * SLOT;
  const int r16 = lane & 15, k4 = lane >> 4;
  dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int ks = 0; ks < SLOT; ks += 4)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[r16][ks + k4], UP[(ks + k4) * SLOT + r16], acc, 0, 0, 0);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = r0 + k4 + 4 * v, gj = ip[r16];
    if (row < l && gj >= 0) vp.V[blk(nb, gj, row)] = acc[v];
  }
}

// A <- G^T A G for one round.  Workgroup (x, y) has four wavefronts; wavefront w takes the A tile (P = y,
// Q = 4 x + w) when Q <= P: A_PQ <- U_P^T A_PQ U_Q (on the lower storage).  A pair without rotations (flag 0) acts as the identity, so its U is not
// read; a tile with nothing to rotate does no loads.  Each 16x16 product is four v_mfma_f64_16x16x4f64 steps
// (accumulator lane L holds rows L/16 + 4v, v = 0..3, of column L%16).  The barriers are uniform over the
// four wavefronts.  (V's update runs in the next round's pair-solve launch.)
__global__ __launch_bounds__(256) void apply_kernel(int l, int np, double* __restrict__ A, int round, int nb,
                                                    const int2* __restrict__ list, const double* __restrict__ Ub,
                                                    const int* __restrict__ flag) {
  __shared__ double Ms[4][SLOT][SLOT + 1];
  __shared__ double Ts[4][SLOT][SLOT + 1];
  __shared__ int ips[4][SLOT], iqs[4][SLOT];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int P = blockIdx.y;
  const int item = (int)blockIdx.x * 4 + wv;
  const bool isA = item <= P && item < np;  // tiles Q <= P: their transposes hold the same stored entries
  const bool fP = flag[P] != 0;
  const bool fQ = isA && flag[item] != 0;
  const bool act = isA && (fP || fQ);
  double (*M)[SLOT + 1] = Ms[wv];
  double (*T)[SLOT + 1] = Ts[wv];
  int* ip = ips[wv];
  int* iq = iqs[wv];
  const int2 pp = get_pair(round, nb, list, P);
  if (lane < SLOT) {
    ip[lane] = pair_slot_index(pp.x, pp.y, lane, l);
    if (isA) {
      const int2 qq = get_pair(round, nb, list, item);
      iq[lane] = pair_slot_index(qq.x, qq.y, lane, l);
    }
  }
  __syncthreads();
  if (act) {
    double mv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = lane + 64 * q, i = u >> 4, j = u & 15;
      const int gi = ip[i], gj = iq[j];
      mv[q] = (gi >= 0 && gj >= 0) ? A[sym(nb, gi, gj)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = lane + 64 * q;
      M[u >> 4][u & 15] = mv[q];
    }
  }
  __syncthreads();
  const int r16 = lane & 15, k4 = lane >> 4;
  const double* UP = Ub + (long long)P * SLOT * SLOT;
  if (act) {
    if (fQ) {
      const double* UQ = Ub + (long long)item * SLOT * SLOT;
      dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < SLOT; ks += 4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(M[r16][ks + k4], UQ[(ks + k4) * SLOT + r16], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) T[k4 + 4 * v][r16] = acc[v];
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) T[k4 + 4 * v][r16] = M[k4 + 4 * v][r16];
    }
  }
  __syncthreads();
  if (act) {
    dbl4 acc2;
    if (fP) {
      acc2 = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < SLOT; ks += 4)
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(UP[(ks + k4) * SLOT + r16], T[ks + k4][r16], acc2, 0, 0, 0);
    } else {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc2[v] = T[k4 + 4 * v][r16];
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int gi = ip[k4 + 4 * v], gj = iq[r16];
      // each stored entry belongs to one tile: (P, Q) with P > Q, or the diagonal tile's lower blocks
      if (gi >= 0 && gj >= 0 && (P != item || (gi >> 3) >= (gj >> 3))) A[sym(nb, gi, gj)] = acc2[v];
    }
  }
}

// ---- one launch per round (full tournament sweeps) -------------------------------------------------------------
// (pair index, half) of block b in tournament round r: the inverse of round_pair.
__device__ __forceinline__ int2 pair_of_block(int r, int b, int nb) {
  const int m = nb - 1, np = nb / 2;
  if (b == m) return make_int2(0, 0);
  if (b == r) return make_int2(0, 1);
  int d = b - r;
  if (d < 0) d += m;  // 1 .. m - 1
  return d <= np - 1 ? make_int2(d, 0) : make_int2(m - d, 1);
}

// Launch q of a sweep with A double-buffered.  Ain holds A before the rotations G of round q - 1 (prev; none at
// the sweep's first round), and the launch
//   * solves the pairs of round q (workgroups [0, npw)) on the subproblems of A' = G^T Ain G: the 16 indices of
//     a new pair come from two blocks, each the half (ha, hb) of a pair Pa, Pb of round q - 1, so with the 32
//     indices of Pa and Pb and W (32 x 16) holding U_Pa's columns of half ha and U_Pb's of half hb,
//     S = W^T (M W), M = Ain on those 32 indices;
//   * writes A' into Aout tile by tile (workgroups [npw, npw + naw), 2 x 2 tiles each, P >= Q: tile (P, Q) <-
//     U_P^T Ain_PQ U_Q on A's stored lower blocks; Aout == Ain only when there are no pair solves);
//   * applies V <- V G (the remaining workgroups, one (pair, 64-column slab of V^T) item each: V is stored
//     transposed, so that the update reads and writes row segments of 16 columns).
// None of the three reads what another writes, so a round costs one launch instead of two.  Every workgroup is
// one wavefront.  Every pair solve writes its U (the identity when it rotated nothing), so the products need no
// flags, and with the block padding in storage no access needs a guard: the loads and stores are unconditional
// (edge tiles of an odd pair count aside).  The products run on v_mfma_f64_16x16x4f64 with operands loaded straight from memory: the
// A operand of step ks on lane (k4 = L/16, r16 = L%16) is X[r16][ks + k4], the B operand Y[ks + k4][r16], and
// the accumulator's v-th value is D[k4 + 4 v][r16], which is exactly the B operand of step ks = 4 v of a second
// product, so T = X Y feeds Z^T T without leaving registers.
struct RoundArgs {
  int l, nb, np;
  int round, npw;  // this round's pair solves (npw = 0: none)
  int prev, naw;   // the previous round (-1: none) and the apply workgroups (g (g + 1) / 2, g = ceil(np / 2); or 0)
  int nvw;         // V items (np * ceil(8 nb / 64), or 0)
  int vmode;       // V's update: 1 by the previous round, 2 by the two previous rounds at once (Uprev2, Uprev)
  const double* Ain;
  double* Aout;
  const double* Uprev;
  const double* Uprev2;  // rotations of round prev - 1 (vmode 2)
  double* Uout;
  const double* Vin;     // V^T before the update and after it (equal only with vmode 1)
  double* Vout;
  const double* thresh_ptr;
  int max_inner, within;
  int delay;  // s_sleep periods (64 clocks each) before the update workgroups start (see launch_sweep_fused)
  int agroup; // tiles per side of a tile group of A's update (1 or 2)
  int prio;   // 1: the pair solves raise their wave priority
};

// Tiles (P0 + i, Q0 + j), i, j < G, of the previous round's pairs with P >= Q (group (gp, gq), gp >= gq, of the
// lower triangle of G x G tile groups): U_P and U_Q are loaded once for G tiles.  With only A's lower blocks
// stored, tile (P, Q), P > Q, owns the stored copies of all its entries (its transpose is not computed) and a
// diagonal tile its lower blocks, so every stored entry is read and written once, by one wavefront (also in place,
// in the tail).
template <int G>
__device__ __forceinline__ void apply_tiles(const RoundArgs& a, int wg, int r16, int k4) {
  int gp = (int)((sqrt(8.0 * wg + 1.0) - 1.0) * 0.5);
  while ((gp + 1) * (gp + 2) / 2 <= wg) ++gp;
  while (gp * (gp + 1) / 2 > wg) --gp;
  const int gq = wg - gp * (gp + 1) / 2;
  const int P0 = G * gp, Q0 = G * gq;
  int2 pp[G], qq[G];
  bool lp[G], lq[G];
  double up[G][4], uq[G][4];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    lp[i] = P0 + i < a.np;
    lq[i] = Q0 + i < a.np;
    const int P = lp[i] ? P0 + i : P0, Q = lq[i] ? Q0 + i : Q0;
    pp[i] = round_pair(a.prev, P, a.nb);
    qq[i] = round_pair(a.prev, Q, a.nb);
    const double* UP = a.Uprev + (long long)P * SLOT * SLOT;
    const double* UQ = a.Uprev + (long long)Q * SLOT * SLOT;
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      up[i][s4] = UP[(4 * s4 + k4) * SLOT + r16];
      uq[i][s4] = UQ[(4 * s4 + k4) * SLOT + r16];
    }
  }
  double mv[G][G][4];
  bool run[G][G];
#pragma unroll
  for (int i = 0; i < G; ++i) {
    const int ipr = slot_index(pp[i], r16);  // row r16 of the tile
#pragma unroll
    for (int j = 0; j < G; ++j) {
      run[i][j] = lp[i] && lq[j] && P0 + i >= Q0 + j;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int gi = slot_index(qq[j], 4 * s4 + k4);  // column 4 s4 + k4 of the tile
        mv[i][j][s4] = run[i][j] ? a.Ain[sym(a.nb, gi, ipr)] : 0.0;
      }
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i)
#pragma unroll
    for (int j = 0; j < G; ++j) {
      dbl4 t = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) t = __builtin_amdgcn_mfma_f64_16x16x4f64(mv[i][j][s4], uq[j][s4], t, 0, 0, 0);
      dbl4 y = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) y = __builtin_amdgcn_mfma_f64_16x16x4f64(up[i][s4], t[s4], y, 0, 0, 0);
      if (run[i][j]) {
        const int gj = slot_index(qq[j], r16);
        const bool diag = P0 + i == Q0 + j;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gr = slot_index(pp[i], k4 + 4 * v);
          if (!diag || (gr >> 3) >= (gj >> 3)) a.Aout[sym(a.nb, gr, gj)] = y[v];
        }
      }
    }
}

__global__ __launch_bounds__(64) void round_kernel(RoundArgs a) {
  const int lane = threadIdx.x;
  const int r16 = lane & 15, k4 = lane >> 4;
  int wg = blockIdx.x;
  if (wg < a.npw) {
    // ---- pair solve
    if (a.prio) __builtin_amdgcn_s_setprio(3);
    __shared__ double S[SLOT][SLOT + 1];
    __shared__ double U[SLOT][SLOT + 1];
    __shared__ double2 cs[8];
    const int k = wg;
    const int2 pq = round_pair(a.round, k, a.nb);
    if (a.prev < 0) {
      double sv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = lane + 64 * q, i = u >> 4, j = u & 15;
        sv[q] = a.Ain[sym(a.nb, slot_index(pq, i), slot_index(pq, j))];
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int u = lane + 64 * q;
        S[u >> 4][u & 15] = sv[q];
      }
    } else {
      const int2 ea = pair_of_block(a.prev, pq.x, a.nb), eb = pair_of_block(a.prev, pq.y, a.nb);
      const int2 pa = round_pair(a.prev, ea.x, a.nb), pb = round_pair(a.prev, eb.x, a.nb);
      const double* Ua = a.Uprev + (long long)ea.x * SLOT * SLOT;
      const double* Ub = a.Uprev + (long long)eb.x * SLOT * SLOT;
      // W[4 ks + k4][r16]: the B operand of T = M W and the A operand of S = W^T T
      double wv[8];
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int c = 4 * ks + k4;
        double v = 0.0;
        if (ks < 4) {
          if (r16 < 8) v = Ua[c * SLOT + ea.y * 8 + r16];
        } else {
          if (r16 >= 8) v = Ub[(c - SLOT) * SLOT + eb.y * 8 + r16 - 8];
        }
        wv[ks] = v;
      }
      // M[c][c'] over source indices c < 16 from Pa, c >= 16 from Pb; lane reads M[rb 16 + r16][4 ks + k4]
      double mv[2][8];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        const int gj = rb == 0 ? slot_index(pa, r16) : slot_index(pb, r16);
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) {
          const int c = 4 * ks + k4;
          const int gi = ks < 4 ? slot_index(pa, c) : slot_index(pb, c - SLOT);
          mv[rb][ks] = a.Ain[sym(a.nb, gi, gj)];
        }
      }
      dbl4 t[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        t[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks) t[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(mv[rb][ks], wv[ks], t[rb], 0, 0, 0);
      }
      // S = W^T T: step ks takes T's rows 4 ks .. 4 ks + 3, held as t[ks / 4][ks % 4]
      dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 8; ++ks)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[ks], t[ks >> 2][ks & 3], acc, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) S[k4 + 4 * v][r16] = acc[v];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int u = lane + 64 * q, i = u >> 4, j = u & 15;
      U[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    jacobi16(S, U, cs, *a.thresh_ptr, a.max_inner, a.within);
    __syncthreads();
    double* Uk = a.Uout + (long long)k * SLOT * SLOT;
    for (int u = lane; u < SLOT * SLOT; u += 64) Uk[u] = U[u >> 4][u & 15];
    return;
  }
  wg -= a.npw;
  for (int d = 0; d < a.delay; ++d) __builtin_amdgcn_s_sleep(1);
  if (wg < a.naw) {
    if (a.agroup == 2) apply_tiles<2>(a, wg, r16, k4);
    else apply_tiles<1>(a, wg, r16, k4);
    return;
  }
  wg -= a.naw;
  if (wg < a.nvw) {
    const int L = a.nb * BSZ;
    const int ns = (L + 63) / 64;
    const int K = wg / ns, c0 = (wg % ns) * 64;
    if (a.vmode == 1) {
      // ---- V <- V G on rows idx_K of V^T (stored transposed): V^T[idx_K, c0 .. c0 + 63] <- U_K^T V^T[idx_K, c0 ..]
      //      (columns past the padded size are not touched)
      const int2 pp = round_pair(a.prev, K, a.nb);
      const double* UP = a.Uprev + (long long)K * SLOT * SLOT;
      double u[4], mv[4][4];
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        u[s4] = UP[(4 * s4 + k4) * SLOT + r16];
        const int gr = slot_index(pp, 4 * s4 + k4);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int col = min(c0 + 16 * cb + r16, L - 1);
          mv[cb][s4] = a.Vin[blk(a.nb, gr, col)];
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(u[s4], mv[cb][s4], acc, 0, 0, 0);
        const int col = c0 + 16 * cb + r16;
        if (col < L)
#pragma unroll
          for (int v = 0; v < 4; ++v) a.Vout[blk(a.nb, slot_index(pp, k4 + 4 * v), col)] = acc[v];
      }
    } else {
      // ---- V <- V G_b G_c for rounds b = prev - 1 and c = prev at once, out of place.  The two blocks x, x' of
      //      pair K of round c were halves hx, hx' of pairs Px, Px' of round b, so with the 32 rows of Px and Px'
      //      and W (32 x 16) holding U_Px's columns of half hx and U_Px''s of half hx' (as in the pair solves),
      //      V^T[idx_K, :] <- C^T V^T[idx_Px u idx_Px', :] with C = W U_K.  C's accumulator is the A operand of
      //      C^T's steps as it stands (step ks takes C's rows 4 ks .. 4 ks + 3).  Each block of V^T is read by
      //      the two pairs of round c that hold its round-b pair's blocks, and written once.
      const int b = a.prev - 1;
      const int2 pk = round_pair(a.prev, K, a.nb);
      const int2 ea = pair_of_block(b, pk.x, a.nb), eb = pair_of_block(b, pk.y, a.nb);
      const int2 pa = round_pair(b, ea.x, a.nb), pb = round_pair(b, eb.x, a.nb);
      const double* Ua = a.Uprev2 + (long long)ea.x * SLOT * SLOT;
      const double* Ub = a.Uprev2 + (long long)eb.x * SLOT * SLOT;
      const double* UK = a.Uprev + (long long)K * SLOT * SLOT;
      // W[16 rb + r16][4 s4 + k4] is nonzero for rb = 0, s4 < 2 (U_Px) and rb = 1, s4 >= 2 (U_Px')
      double w0[2], w1[2], uk[4];
#pragma unroll
      for (int s4 = 0; s4 < 2; ++s4) {
        w0[s4] = Ua[r16 * SLOT + ea.y * 8 + 4 * s4 + k4];
        w1[s4] = Ub[r16 * SLOT + eb.y * 8 + 4 * s4 + k4];
      }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) uk[s4] = UK[(4 * s4 + k4) * SLOT + r16];
      dbl4 c[2];
      c[0] = dbl4{0.0, 0.0, 0.0, 0.0};
      c[1] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s4 = 0; s4 < 2; ++s4) {
        c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(w0[s4], uk[s4], c[0], 0, 0, 0);
        c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(w1[s4], uk[2 + s4], c[1], 0, 0, 0);
      }
      double mv[4][8];
#pragma unroll
      for (int ks = 0; ks < 8; ++ks) {
        const int cr = 4 * ks + k4;
        const int gr = ks < 4 ? slot_index(pa, cr) : slot_index(pb, cr - SLOT);
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          const int col = min(c0 + 16 * cb + r16, L - 1);
          mv[cb][ks] = a.Vin[blk(a.nb, gr, col)];
        }
      }
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        dbl4 acc = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < 8; ++ks)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(c[ks >> 2][ks & 3], mv[cb][ks], acc, 0, 0, 0);
        const int col = c0 + 16 * cb + r16;
        if (col < L)
#pragma unroll
          for (int v = 0; v < 4; ++v) a.Vout[blk(a.nb, slot_index(pk, k4 + 4 * v), col)] = acc[v];
      }
    }
  }
}

// Sums of squares of A over the BSZ x BSZ blocks (b1, b2 >= b1): off-diagonal entries (boff), all entries,
// doubled off the block diagonal for the mirrored block (ball), and per diagonal block the number of positive
// diagonal entries (bpos); the diagonal itself goes to dg.  Workgroup (chunk, b1): the BSZ rows of block row b1
// over 256 consecutive columns, one column per thread, so every row segment is one coalesced 2 KB read.
// Warm-basis check without the second product: with V = Z P0 and d_i = P0_i . V_i (the diagonal of
// A = P0^T Z P0), off(A) = |V - P0 diag(d)|_F and |A|_F = |V|_F for orthogonal P0.  Workgroup r sums row r
// (fixed tree) into out[r], out[l + r], and flags d_r > 0 in out[2 l + r].
__global__ __launch_bounds__(256) void warm_check_kernel(int l, const double* __restrict__ P0,
                                                         const double* __restrict__ V, const double* __restrict__ d,
                                                         double* __restrict__ out) {
  __shared__ double so_s[256], sa_s[256];
  const int r = blockIdx.x, t = threadIdx.x;
  double so = 0.0, sa = 0.0;
  for (int i = t; i < l; i += 256) {
    const double v = V[(long long)r * l + i];
    const double e = v - P0[(long long)r * l + i] * d[i];
    so += e * e;
    sa += v * v;
  }
  so_s[t] = so;
  sa_s[t] = sa;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      so_s[t] += so_s[t + h];
      sa_s[t] += sa_s[t + h];
    }
    __syncthreads();
  }
  if (t == 0) {
    out[r] = so_s[0];
    out[l + r] = sa_s[0];
    out[2 * l + r] = d[r] > 0.0 ? 1.0 : 0.0;
  }
}

__global__ __launch_bounds__(256) void block_norm_kernel(int l, int nb, const double* __restrict__ A,
                                                         double* __restrict__ boff, double* __restrict__ ball,
                                                         double* __restrict__ bpos, double* __restrict__ dg) {
  const int b1 = blockIdx.y;
  if ((int)blockIdx.x * (256 / BSZ) + (256 / BSZ) - 1 < b1) return;  // the chunk lies left of the diagonal
  const int t = threadIdx.x;
  const int j = blockIdx.x * 256 + t;
  const int b2 = j / BSZ;
  const bool need = b2 >= b1 && b2 < nb;
  double v[BSZ];
#pragma unroll
  for (int r = 0; r < BSZ; ++r) {
    const int i = b1 * BSZ + r;
    v[r] = (need && i < l && j < l) ? A[sym(nb, i, j)] : 0.0;
  }
  double off = 0.0, all = 0.0, pos = 0.0;
#pragma unroll
  for (int r = 0; r < BSZ; ++r) {
    const double sq = v[r] * v[r];
    all += sq;
    if (b1 * BSZ + r != j) {
      off += sq;
    } else {
      pos = v[r] > 0.0 ? 1.0 : 0.0;
      if (j < l) dg[j] = v[r];
    }
  }
#pragma unroll
  for (int o = 1; o < BSZ; o <<= 1) {  // the BSZ lanes of one block column are consecutive
    off += __shfl_xor(off, o);
    all += __shfl_xor(all, o);
    pos += __shfl_xor(pos, o);
  }
  if ((t & (BSZ - 1)) == 0 && need) {
    boff[(long long)b1 * nb + b2] = off;
    ball[(long long)b1 * nb + b2] = (b1 < b2 ? 2.0 : 1.0) * all;
    if (b1 == b2) bpos[b1] = pos;
  }
}

// Ascending order of the diagonal dg by ranks: element i goes to position #{j : k_j < k_i, or k_j == k_i and
// j < i} (keys ordered totally, NaN as +inf, so the positions are a permutation); w[rank] = value, perm[rank] =
// index.  Workgroup b ranks elements 16 b .. 16 b + 15, each counted by 16 threads over a sixteenth of the keys,
// staged in LDS (l <= 4096).
__global__ __launch_bounds__(256) void rank_sort_kernel(int l, const double* __restrict__ dg, double* __restrict__ w,
                                                        int* __restrict__ perm) {
  __shared__ double key[4096];
  __shared__ int cnt[16][16];
  const int t = threadIdx.x;
  for (int j0 = 0; j0 < l; j0 += 4 * 256) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + t + 256 * q;
      v[q] = (j < l) ? dg[j] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + t + 256 * q;
      if (j < l) key[j] = isnan(v[q]) ? INFINITY : v[q];
    }
  }
  __syncthreads();
  const int il = t & 15, part = t >> 4;
  const int i = blockIdx.x * 16 + il;
  const double ki = (i < l) ? key[i] : 0.0;
  const int per = (l + 15) / 16;
  const int jb = part * per, je = min(l, jb + per);
  int c = 0;
  int j = jb;
  for (; j + 8 <= je; j += 8) {
    double kj[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) kj[q] = key[j + q];
#pragma unroll
    for (int q = 0; q < 8; ++q) c += (kj[q] < ki || (kj[q] == ki && j + q < i)) ? 1 : 0;
  }
  for (; j < je; ++j) {
    const double kj = key[j];
    c += (kj < ki || (kj == ki && j < i)) ? 1 : 0;
  }
  cnt[part][il] = c;
  __syncthreads();
  if (t < 16 && i < l) {
    int r = 0;
#pragma unroll
    for (int p = 0; p < 16; ++p) r += cnt[p][il];
    w[r] = dg[i];
    perm[r] = i;
  }
}

__global__ void permute_cols_kernel(int l, const double* __restrict__ V, const int* __restrict__ perm, double* __restrict__ P) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  P[u] = V[(long long)i * l + perm[j]];
}

// P[i][j] = V[i][perm[j]] = Vt[perm[j]][i] with Vt = V^T in blocked storage: 32 x 32 tiles of P through LDS
// (row segments of Vt in, row segments of P out).
__global__ __launch_bounds__(256) void permute_cols_blocked_kernel(int l, int nb, const double* __restrict__ Vt,
                                                                   const int* __restrict__ perm, double* __restrict__ P) {
  __shared__ double T[32][33];
  const int i0 = blockIdx.y * 32, j0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int jj = ty; jj < 32; jj += 8) {
    const int j = j0 + jj, i = i0 + tx;
    T[jj][tx] = (j < l && i < l) ? Vt[blk(nb, perm[j], i)] : 0.0;
  }
  __syncthreads();
  for (int ii = ty; ii < 32; ii += 8) {
    const int i = i0 + ii, j = j0 + tx;
    if (i < l && j < l) P[(long long)i * l + j] = T[tx][ii];
  }
}

// Blocked storage of the row-major l x l X (ld l), or of X^T with trans, zeros past l (X null: the identity).
// One thread per stored entry, in storage order.
__global__ void to_blocked_kernel(int l, int nb, const double* __restrict__ X, int trans, double* __restrict__ B) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)nb * nb * 64) return;
  const long long b = u >> 6;
  const int e = (int)(u & 63);
  const int i = (int)(b / nb) * 8 + (e >> 3), j = (int)(b % nb) * 8 + (e & 7);
  double v = 0.0;
  if (i < l && j < l) v = X ? (trans ? X[(long long)j * l + i] : X[(long long)i * l + j]) : (i == j ? 1.0 : 0.0);
  B[u] = v;
}

}  // namespace

struct EigWork {
  int lmax = 0;
  // set for the allocation-free entry point: every device buffer below lies in the static scratch array, hb is
  // plain host memory filled by a copy after each block-norm pass, the threshold goes up by a fill kernel, and
  // sweeps are always full tournaments launched directly (no graph, no threshold schedule)
  bool noalloc = false;
  // one captured full-tournament sweep (all rounds) per (l, A/V buffers); replayed with hipGraphLaunch
  int graph_l = -1;
  int graph_inner = -1;
  const double* graph_tmp = nullptr;
  hipGraphExec_t graph = nullptr;
  bool graph_failed = false;
  double* U = nullptr;        // device [3][npairs_max * 256]: rotations of the last rounds (round q in q mod 2 or
                              // q mod 3)
  int* flag = nullptr;        // device [2][npairs_max]
  int* perm = nullptr;        // device [lmax]
  double* dg = nullptr;       // device [lmax]: the diagonal of A at the last block-norm pass
  double* hb = nullptr;       // block norms: off-diagonal part [nbmax^2], all entries [nbmax^2], positive diagonal
                              // counts [nbmax]; pinned, mapped and coherent host memory written by the kernel
  double* boff = nullptr;     // device address of hb
  // uploads: [0] the rotation threshold, [2..] the pair lists of a threshold sweep [(nbmax - 1) * nbmax / 2];
  // device copy, host staging (pinned, mapped and coherent) and its device address, copied by a kernel
  double* up = nullptr;
  double* hup = nullptr;
  double* hup_dev = nullptr;
  int2* list = nullptr;       // up + 2
  int2* hlist = nullptr;      // hup + 2
  double* wh = nullptr;       // mapped host: per-row sums of the warm-basis check (3 lmax)
  double* wdev = nullptr;     // its device alias
  std::vector<int> round_k;   // active pairs per round of the current threshold sweep
};
static int block_count(int l) {
  int nb = (l + BSZ - 1) / BSZ;
  if (nb < 2) nb = 2;
  if (nb & 1) ++nb;
  return nb;
}

EigWork* eig_work_create(int lmax) {
  EigWork* w = new EigWork();
  w->lmax = lmax;
  const int nbmax = block_count(lmax);
  const int npm = nbmax / 2;
  const size_t nb2 = (size_t)nbmax * nbmax;
  const size_t nlist = (size_t)(nbmax - 1) * npm;
  bool ok = hipMalloc(&w->U, sizeof(double) * (size_t)npm * 256 * 3) == hipSuccess &&
            hipMalloc(&w->flag, sizeof(int) * (size_t)npm * 2) == hipSuccess &&
            hipMalloc(&w->perm, sizeof(int) * (size_t)lmax) == hipSuccess &&
            hipMalloc(&w->dg, sizeof(double) * (size_t)lmax) == hipSuccess &&
            hipHostMalloc(&w->hb, sizeof(double) * (2 * nb2 + nbmax), hipHostMallocMapped | hipHostMallocCoherent) ==
                hipSuccess &&
            hipHostGetDevicePointer(reinterpret_cast<void**>(&w->boff), w->hb, 0) == hipSuccess &&
            hipMalloc(&w->up, sizeof(double) * (2 + nlist)) == hipSuccess &&
            hipHostMalloc(&w->hup, sizeof(double) * (2 + nlist), hipHostMallocMapped | hipHostMallocCoherent) ==
                hipSuccess &&
            hipHostGetDevicePointer(reinterpret_cast<void**>(&w->hup_dev), w->hup, 0) == hipSuccess &&
            hipHostMalloc(&w->wh, sizeof(double) * 3 * (size_t)lmax, hipHostMallocMapped | hipHostMallocCoherent) ==
                hipSuccess &&
            hipHostGetDevicePointer(reinterpret_cast<void**>(&w->wdev), w->wh, 0) == hipSuccess;
  if (!ok) { eig_work_destroy(w); return nullptr; }
  static_assert(sizeof(int2) == sizeof(double), "pair lists travel as doubles");
  w->list = reinterpret_cast<int2*>(w->up + 2);
  w->hlist = reinterpret_cast<int2*>(w->hup + 2);
  return w;
}

void eig_work_destroy(EigWork* w) {
  if (!w) return;
  if (w->graph) hipGraphExecDestroy(w->graph);
  hipFree(w->U); hipFree(w->flag); hipFree(w->perm); hipFree(w->dg);
  hipHostFree(w->hb); hipFree(w->up); hipHostFree(w->hup); hipHostFree(w->wh);
  delete w;
}

// Block norms of A to the host; returns off(A), |A|_F (sums in a fixed order on the host) and the number of
// positive diagonal entries.
static hipError_t block_norms(EigWork* w, int l, int nb, const double* A, hipStream_t st, double* off, double* all,
                              int* npos) {
  const size_t nb2 = (size_t)nb * nb;
  hipLaunchKernelGGL(block_norm_kernel, dim3((nb * BSZ + 255) / 256, nb), dim3(256), 0, st, l, nb, A, w->boff,
                     w->boff + nb2, w->boff + 2 * nb2, w->dg);
  KOT_HIP_TRY(hipGetLastError());
  if (w->noalloc)
    KOT_HIP_TRY(hipMemcpyAsync(w->hb, w->boff, sizeof(double) * (2 * nb2 + nb), hipMemcpyDeviceToHost, st));
  KOT_HIP_TRY(hipStreamSynchronize(st));
  double so = 0.0, sa = 0.0, sp = 0.0;
  for (int b1 = 0; b1 < nb; ++b1) {
    for (int b2 = b1; b2 < nb; ++b2) {
      const size_t u = (size_t)b1 * nb + b2;
      so += (b2 > b1 ? 2.0 : 1.0) * w->hb[u];
      sa += w->hb[nb2 + u];
    }
    sp += w->hb[2 * nb2 + b1];
  }
  *off = std::sqrt(so);
  *all = std::sqrt(sa);
  *npos = (int)sp;
  return hipSuccess;
}

// Threshold sweep schedule: block pairs whose off-diagonal norm exceeds tau (and blocks with internal
// off-diagonal mass) are packed greedily, largest first, into rounds of disjoint pairs; each round is then
// completed to a partition of all blocks by pairs that rotate nothing.  Returns false (no schedule) when the
// active set is too large for this to beat the full tournament.
static bool threshold_schedule(EigWork* w, int nb, double tau2) {
  const size_t nb2 = (size_t)nb * nb;
  struct E { double v; int a, b; };
  std::vector<E> edges;
  std::vector<char> self(nb, 0);
  for (int b1 = 0; b1 < nb; ++b1) {
    if (w->hb[(size_t)b1 * nb + b1] > tau2) self[b1] = 1;
    for (int b2 = b1 + 1; b2 < nb; ++b2) {
      const double v = w->hb[(size_t)b1 * nb + b2];
      if (v > tau2) edges.push_back({v, b1, b2});
    }
  }
  const int np = nb / 2, maxr = nb - 1;
  if ((long long)edges.size() > (long long)np * maxr / 4) return false;
  std::stable_sort(edges.begin(), edges.end(), [](const E& x, const E& y) { return x.v > y.v; });
  std::vector<std::vector<char>> used;
  std::vector<std::vector<int2>> rounds;
  std::vector<char> covered(nb, 0);
  auto place = [&](int a, int b) -> bool {
    size_t r = 0;
    while (r < rounds.size() && (used[r][a] || used[r][b])) ++r;
    if (r == rounds.size()) {
      if ((int)r >= maxr / 2) return false;
      rounds.emplace_back();
      used.emplace_back(nb, 0);
    }
    rounds[r].push_back(make_int2(a, b));
    used[r][a] = used[r][b] = 1;
    covered[a] = covered[b] = 1;
    return true;
  };
  for (const E& e : edges)
    if (!place(e.a, e.b)) return false;
  for (int b = 0; b < nb; ++b) {
    if (!self[b] || covered[b]) continue;
    // pair b with the first block free in the first round where b is free (another uncovered block if any)
    size_t r = 0;
    while (r < rounds.size() && used[r][b]) ++r;
    int partner = -1;
    if (r < rounds.size()) {
      for (int c = 0; c < nb && partner < 0; ++c)
        if (c != b && !used[r][c] && self[c] && !covered[c]) partner = c;
      for (int c = 0; c < nb && partner < 0; ++c)
        if (c != b && !used[r][c]) partner = c;
    } else {
      for (int c = 0; c < nb && partner < 0; ++c)
        if (c != b && self[c] && !covered[c]) partner = c;
      if (partner < 0) partner = (b == 0) ? 1 : 0;
    }
    if (!place(std::min(b, partner), std::max(b, partner))) return false;
  }
  if (rounds.empty()) return false;
  w->round_k.assign(rounds.size(), 0);
  for (size_t r = 0; r < rounds.size(); ++r) {
    int2* dst = w->hlist + r * np;
    int k = 0;
    for (const int2& pr : rounds[r]) dst[k++] = pr;
    w->round_k[r] = k;
    int pending = -1;
    for (int b = 0; b < nb; ++b) {
      if (used[r][b]) continue;
      if (pending < 0) pending = b;
      else { dst[k++] = make_int2(pending, b); pending = -1; }
    }
  }
  (void)nb2;
  return true;
}

size_t eig_mat_doubles(int l) {
  const size_t L = (size_t)block_count(l) * BSZ;
  return L * L;
}

hipError_t eigh_jacobi(EigWork* w, int l, const double* Z, const double* P0, double* P, double* wv, double* tmp,
                       int tmp_mats, int max_sweeps, int inner_sweeps, double tol, int* sweeps, double* rel_off,
                       int* npos, hipStream_t st) {
  if (l > w->lmax || (w->noalloc && P0) || tmp_mats < 2 || (P0 && tmp_mats < 3)) return hipErrorInvalidValue;
  const int nb = block_count(l);
  const long long mat = (long long)eig_mat_doubles(l);
  double* A = tmp;                                    // blocked A
  double* V = tmp + mat;                              // blocked V^T (row-major staging before the sweeps)
  double* A2 = tmp_mats >= 3 ? tmp + 2 * mat : nullptr;  // second blocked A (row-major staging before the sweeps)
  double* V2 = tmp_mats >= 4 ? tmp + 3 * mat : nullptr;  // second V^T: V's update by two rounds at once
  const long long nn = (long long)l * l;
  const int eb = (int)((nn + 255) / 256);
  const int ebb = (int)((mat + 255) / 256);
  // ascending eigenvalues from w->dg and the columns of the basis permuted to match into P: src row-major, or
  // the blocked V when src is null
  auto finish = [&](const double* src) -> hipError_t {
    if (l > 4096) return hipErrorInvalidValue;
    hipLaunchKernelGGL(rank_sort_kernel, dim3((l + 15) / 16), dim3(256), 0, st, l, w->dg, wv, w->perm);
    KOT_HIP_TRY(hipGetLastError());
    if (src) hipLaunchKernelGGL(permute_cols_kernel, dim3(eb), dim3(256), 0, st, l, src, w->perm, P);
    else hipLaunchKernelGGL(permute_cols_blocked_kernel, dim3((l + 31) / 32, (l + 31) / 32), dim3(256), 0, st, l, nb,
                            V, w->perm, P);
    return hipGetLastError();
  };
  if (P0) {
    // A = P0^T Z P0 (Z P0 staged row-major in V's region, the product row-major in A2's; P0 may alias the output
    // P), then both to blocked storage: A from the product, V from P0
    GemmArgs g{};
    g.transa = 0; g.transb = 0; g.m = l; g.n = l; g.k = l; g.alpha = 1.0; g.beta = 0.0;
    g.A = Z; g.lda = l; g.B = P0; g.ldb = l; g.C = V; g.ldc = l; g.batch = 1;
    KOT_HIP_TRY(gemm_f64(g, st));
    if (l >= kDiagParts) {
      // Once the iteration settles the warm basis often diagonalizes Z to the tolerance already: test that from
      // V alone (A's buffer serves as the column dots' workspace) and skip the second product and the sweeps.
      KOT_HIP_TRY(diag_dot(0, l, l, 1.0, P0, l, V, l, 0.0, w->dg, A, st));
      hipLaunchKernelGGL(warm_check_kernel, dim3(l), dim3(256), 0, st, l, P0, V, w->dg, w->wdev);
      KOT_HIP_TRY(hipGetLastError());
      KOT_HIP_TRY(hipStreamSynchronize(st));
      double so = 0.0, sa = 0.0, sp = 0.0;
      for (int r = 0; r < l; ++r) {
        so += w->wh[r];
        sa += w->wh[l + r];
        sp += w->wh[2 * l + r];
      }
      if (std::sqrt(so) <= tol * std::sqrt(sa)) {
        if (P0 == P) KOT_HIP_TRY(vec_copy((int)nn, P0, V, st));  // the permutation cannot run in place
        *sweeps = 0;
        *rel_off = (sa > 0.0) ? std::sqrt(so) / std::sqrt(sa) : 0.0;
        if (npos) *npos = (int)sp;
        return finish(P0 == P ? V : P0);
      }
    }
    g.transa = 1; g.A = P0; g.B = V; g.C = A2;
    g.lower = 1; g.mirror = 1;  // symmetric result: lower tiles, mirrored
    KOT_HIP_TRY(gemm_f64(g, st));
    hipLaunchKernelGGL(to_blocked_kernel, dim3(ebb), dim3(256), 0, st, l, nb, A2, 0, A);
    KOT_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(to_blocked_kernel, dim3(ebb), dim3(256), 0, st, l, nb, P0, 1, V);
    KOT_HIP_TRY(hipGetLastError());
  } else {
    // Z may lie in V's region (the allocation-free path stages it there): it is read before V is written
    hipLaunchKernelGGL(to_blocked_kernel, dim3(ebb), dim3(256), 0, st, l, nb, Z, 0, A);
    KOT_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(to_blocked_kernel, dim3(ebb), dim3(256), 0, st, l, nb, nullptr, 0, V);
    KOT_HIP_TRY(hipGetLastError());
  }
  const int np = nb / 2;
  const int nslab = (l + SLOT - 1) / SLOT;
  double off = 0.0, all = 0.0;
  int pos = 0;
  KOT_HIP_TRY(block_norms(w, l, nb, A, st, &off, &all, &pos));
  int s = 0;
  const double thresh_rel = 1e-18;
  // Round q of a sweep (rotations in buffer q & 1): the pair solves of round q together with V's update by
  // round q - 1, then A's update by round q; after the last round, V's update by it.
  const int nvwg = (np * nslab + 3) / 4;
  double* Ub[2] = {w->U, w->U + (size_t)(block_count(w->lmax) / 2) * SLOT * SLOT};
  int* Fb[2] = {w->flag, w->flag + block_count(w->lmax) / 2};
  auto vprev = [&](int q, int r_prev, const int2* list_prev) {
    VPrev vp{};
    vp.active = q > 0 ? 1 : 0;
    vp.round = r_prev; vp.list = list_prev; vp.U = Ub[(q - 1) & 1]; vp.flag = Fb[(q - 1) & 1]; vp.V = V;
    vp.nslab = nslab;
    return vp;
  };
  auto launch_round = [&](hipStream_t s_, int q, int r, const int2* list, int kact, int r_prev,
                          const int2* list_prev) -> hipError_t {
    const int within = (list != nullptr || r == 0) ? 1 : 0;
    hipLaunchKernelGGL(pair_solve_kernel, dim3(np + (q > 0 ? nvwg : 0)), dim3(64), 0, s_, l, A, r, nb, list, kact,
                       np, Ub[q & 1], Fb[q & 1], w->up, inner_sweeps, within, vprev(q, r_prev, list_prev), np);
    KOT_HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(apply_kernel, dim3((np + 3) / 4, np), dim3(256), 0, s_, l, np, A, r, nb, list, Ub[q & 1],
                       Fb[q & 1]);
    return hipGetLastError();
  };
  auto launch_v_tail = [&](hipStream_t s_, int q_last, int r_last, const int2* list_last) -> hipError_t {
    hipLaunchKernelGGL(pair_solve_kernel, dim3(nvwg), dim3(64), 0, s_, l, A, 0, nb, nullptr, 0, 0, Ub[0], Fb[0],
                       w->up, inner_sweeps, 1, vprev(q_last + 1, r_last, list_last), np);
    return hipGetLastError();
  };
  // With a second buffer for A, round q's pair solves, A's update by round q - 1 (Ain = buffer (q - 1) & 1 ->
  // buffer q & 1) and V's update by round q - 1 share launch q (round_kernel); a tail launch applies the last
  // round to A (into the first buffer, in place when that is where A is) and to V.
  // V's update: with a second V buffer, even launches q = 2, 4, .. apply rounds q - 2 and q - 1 at once (out of
  // place, V^T read twice and written once per two rounds) and the tail the rounds left; otherwise launch q
  // applies round q - 1 in place.  V ends every sweep in its first buffer (an odd number of buffer flips is
  // undone by an out-of-place tail, or by a copy).
  auto launch_sweep_fused = [&](hipStream_t s_) -> hipError_t {
    const int R = nb - 1;
    double* Abuf[2] = {A, A2};
    double* Vb[2] = {V, V2};
    double* Ub3[3] = {w->U, w->U + (size_t)(block_count(w->lmax) / 2) * SLOT * SLOT,
                      w->U + 2 * (size_t)(block_count(w->lmax) / 2) * SLOT * SLOT};
    const bool pairs2 = V2 != nullptr;
    int cur = 0;  // the V buffer holding V before launch q
    for (int q = 0; q <= R; ++q) {
      RoundArgs ra{};
      ra.l = l; ra.nb = nb; ra.np = np;
      ra.round = q; ra.npw = q < R ? np : 0;
      // 2 x 2 tile groups and raised pair-solve priority: 8.05 us per l = 1000 round (single tiles: A's update
      // alone is faster, 4.4 against 5.8 us, but slows the pair solves more, 8.3-8.4 us per round)
      ra.agroup = 2;
      ra.prio = 1;
      const int ng = (np + ra.agroup - 1) / ra.agroup;
      ra.prev = q - 1; ra.naw = q > 0 ? ng * (ng + 1) / 2 : 0;
      ra.Ain = q > 0 ? Abuf[(q - 1) & 1] : A;
      ra.Aout = q < R ? Abuf[q & 1] : A;
      if (pairs2) {
        ra.Uprev = Ub3[(q + 2) % 3];
        ra.Uprev2 = Ub3[(q + 1) % 3];
        ra.Uout = Ub3[q % 3];
      } else {
        ra.Uprev = Ub[(q + 1) & 1];
        ra.Uout = Ub[q & 1];
      }
      ra.vmode = 0;
      if (!pairs2) {
        if (q > 0) ra.vmode = 1;
        ra.Vin = V; ra.Vout = V;
      } else if (q >= 2 && (q & 1) == 0) {
        ra.vmode = 2;  // rounds q - 2, q - 1
        ra.Vin = Vb[cur]; ra.Vout = Vb[cur ^ 1];
        cur ^= 1;
      } else if (q == R) {
        ra.vmode = 1;  // round R - 1 (R odd); out of place when that returns V to its first buffer
        ra.Vin = Vb[cur]; ra.Vout = Vb[0];
        cur = 0;
      }
      ra.nvw = ra.vmode ? np * ((nb * BSZ + 63) / 64) : 0;
      ra.thresh_ptr = w->up;
      ra.max_inner = inner_sweeps; ra.within = q == 0 ? 1 : 0;
      // the update wavefronts hold back about 0.9 us so that the pair solves' loads (the round's critical path)
      // are not queued behind theirs: 8.2 instead of 8.5 us per round at l = 1000
      ra.delay = ra.npw > 0 ? 32 : 0;
      const int grid = ra.npw + ra.naw + ra.nvw;
      hipLaunchKernelGGL(round_kernel, dim3(grid), dim3(64), 0, s_, ra);
      KOT_HIP_TRY(hipGetLastError());
    }
    if (cur != 0) KOT_HIP_TRY(vec_copy((int)mat, Vb[cur], V, s_));
    return hipSuccess;
  };
  auto launch_sweep = [&](hipStream_t s_) -> hipError_t {
    if (A2) return launch_sweep_fused(s_);
    for (int r = 0; r < nb - 1; ++r) KOT_HIP_TRY(launch_round(s_, r, r, nullptr, np, r - 1, nullptr));
    return launch_v_tail(s_, nb - 2, nb - 2, nullptr);
  };
  // flops of one full sweep: per round 2 x 2 x 16^3 per A tile and 2 x 16^3 per V tile
  const double sweep_flops = (double)(nb - 1) * (4.0 * 4096.0 * np * np + 2.0 * 4096.0 * nslab * np);
  // algorithmic bytes of a full sweep: per round A's lower triangle (A is symmetric) read and written once, 8 l^2,
  // and V read and written once per round (16 l^2) or, with the two-round update, once per two rounds (8 l^2)
  const double sweep_bytes = (A2 && V2 ? 16.0 : 24.0) * l * (double)l * (nb - 1);
  const double npairs = 0.5 * nb * (nb + 1.0);
  while (off > tol * all && s < max_sweeps) {
    if (!w->noalloc) w->hup[0] = thresh_rel * all;  // the stream is idle here (block_norms synchronized it)
    Profiler* pf = (g_prof && g_prof->on) ? g_prof : nullptr;
    // threshold sweep over the block pairs above tau; if every pair is at or below tau, then
    // off(A)^2 <= npairs tau^2 = (tol |A|_F / 2)^2, so the stopping test is met
    const double tau2 = 0.25 * tol * tol * all * all / npairs;
    if (w->noalloc) {
      KOT_HIP_TRY(vec_fill(1, thresh_rel * all, w->up, st));
      if (pf) pf->begin(st, PROF_EIG_ROUND, sweep_flops, sweep_bytes);
      KOT_HIP_TRY(launch_sweep(st));
      if (pf) pf->end(st);
    } else if (threshold_schedule(w, nb, tau2)) {
      const int R = (int)w->round_k.size();
      KOT_HIP_TRY(vec_copy(2 + R * np, w->hup_dev, w->up, st));  // threshold and pair lists
      double fl = 0.0, by = 0.0;
      for (int r = 0; r < R; ++r) {
        const double k = w->round_k[r];
        fl += 8192.0 * (2.0 * k * k + 2.0 * k * (np - k) + k * nslab);
        // the active tiles of A (half of them, by symmetry) and V's active slabs, read and written
        by += 2048.0 * ((double)np * np - (np - k) * (np - k)) + 4096.0 * k * nslab;
      }
      if (pf) pf->begin(st, PROF_EIG_ROUND, fl, by);
      for (int r = 0; r < R; ++r)
        KOT_HIP_TRY(launch_round(st, r, 0, w->list + (size_t)r * np, w->round_k[r], 0,
                                 r > 0 ? w->list + (size_t)(r - 1) * np : nullptr));
      KOT_HIP_TRY(launch_v_tail(st, R - 1, 0, w->list + (size_t)(R - 1) * np));
      if (pf) pf->end(st);
    } else {
      KOT_HIP_TRY(vec_copy(2, w->hup_dev, w->up, st));  // threshold
      if (!w->graph_failed &&
          (w->graph == nullptr || w->graph_l != l || w->graph_tmp != tmp || w->graph_inner != inner_sweeps)) {
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
          hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;  // a failed capture must not stay open
          if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
            hipGraph_t g2 = nullptr;
            (void)hipStreamEndCapture(st, &g2);
            if (g2) hipGraphDestroy(g2);
          }
          (void)hipGetLastError();
          w->graph = nullptr;
          w->graph_failed = true;
        } else {
          w->graph_l = l;
          w->graph_tmp = tmp;
          w->graph_inner = inner_sweeps;
        }
      }
      if (pf) pf->begin(st, PROF_EIG_ROUND, sweep_flops, sweep_bytes);
      if (w->graph) KOT_HIP_TRY(hipGraphLaunch(w->graph, st));
      else KOT_HIP_TRY(launch_sweep(st));
      if (pf) pf->end(st);
    }
    ++s;
    KOT_HIP_TRY(block_norms(w, l, nb, A, st, &off, &all, &pos));
  }
  *sweeps = s;
  // a non-finite entry (NaN, or an infinity and the NaNs its rotations make) leaves a non-finite norm: report
  // it as a non-finite ratio, so that the caller does not take the sweeps' output for converged
  if (!std::isfinite(off) || !std::isfinite(all)) *rel_off = NAN;
  else *rel_off = (all > 0.0) ? off / all : 0.0;
  if (npos) *npos = pos;
  return finish(nullptr);
}

// ---- allocation-free eigendecomposition ---------------------------------------------------------------------
// Scratch for eigh_jacobi_noalloc: one static array per device (each GPU the library runs on holds its own copy
// until the process ends), sized for l <= kNoAllocMaxL.  Host code never uses the array's name as an address:
// the device address comes from hipGetSymbolAddress, once per device, with that device current.
namespace {
constexpr int kNoAllocMaxNb = kNoAllocMaxL / BSZ;            // 64 blocks of 8
constexpr int kNoAllocMaxNp = kNoAllocMaxNb / 2;
constexpr size_t kNoAllocDoubles =
    2 * (size_t)kNoAllocMaxL * kNoAllocMaxL                    // A, V
    + 2 * (size_t)kNoAllocMaxNp * SLOT * SLOT                  // U (two rounds)
    + (size_t)kNoAllocMaxL                                     // dg
    + 2 * (size_t)kNoAllocMaxNb * kNoAllocMaxNb + kNoAllocMaxNb  // block norms
    + 32                                                       // threshold slot (up)
    + (size_t)kNoAllocMaxNp + kNoAllocMaxL;                    // flags (two rounds) and ranks (ints, two per double)
constexpr int kNoAllocMaxDevices = 64;
double g_noalloc_hb[2 * kNoAllocMaxNb * kNoAllocMaxNb + kNoAllocMaxNb];  // host copy of the block norms
double* g_noalloc_ptr[kNoAllocMaxDevices] = {};
std::mutex g_noalloc_mu;
}  // namespace

static __device__ __align__(256) double scratch[kNoAllocDoubles];

size_t eigh_noalloc_scratch_bytes() { return sizeof(double) * kNoAllocDoubles; }

// The calling thread's current device must be `device`.
static hipError_t noalloc_scratch(int device, double** out) {
  if (device < 0 || device >= kNoAllocMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[device]) {
    void* ptr = nullptr;
    KOT_HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    g_noalloc_ptr[device] = static_cast<double*>(ptr);
  }
  *out = g_noalloc_ptr[device];
  return hipSuccess;
}

hipError_t eigh_jacobi_noalloc(int device, int l, const double* Z, double* P, double* wv, int max_sweeps,
                               int inner_sweeps, double tol, int* sweeps, double* rel_off, hipStream_t st) {
  if (l < 1 || l > kNoAllocMaxL) return hipErrorInvalidValue;
  double* base = nullptr;
  KOT_HIP_TRY(noalloc_scratch(device, &base));
  const size_t ll = (size_t)kNoAllocMaxL * kNoAllocMaxL;
  double* A = base;                      // A then V (eigh_jacobi's tmp layout: V = tmp + eig_mat_doubles(l))
  double* cur = base + 2 * ll;
  EigWork w;
  w.noalloc = true;
  w.graph_failed = true;
  w.lmax = kNoAllocMaxL;
  w.U = cur;    cur += 2 * (size_t)kNoAllocMaxNp * SLOT * SLOT;
  w.dg = cur;   cur += kNoAllocMaxL;
  w.boff = cur; cur += 2 * (size_t)kNoAllocMaxNb * kNoAllocMaxNb + kNoAllocMaxNb;
  w.up = cur;   cur += 32;
  w.flag = reinterpret_cast<int*>(cur);
  w.perm = w.flag + 2 * kNoAllocMaxNp;
  w.hb = g_noalloc_hb;
  // the symmetrized input is staged row-major in V's region, from which eigh_jacobi forms the blocked A
  double* Zs = A + eig_mat_doubles(l);
  KOT_HIP_TRY(form_z(l, Z, 0.0, Z, 0.0, Zs, st));
  int npos = 0;
  return eigh_jacobi(&w, l, Zs, nullptr, P, wv, A, 2, max_sweeps, inner_sweeps, tol, sweeps, rel_off, &npos, st);
}

}  // namespace kot
