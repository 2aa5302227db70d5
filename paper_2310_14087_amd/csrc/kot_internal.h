// Internal declarations shared by the HIP kernels and the host orchestration of libkotssn.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>
#include <vector>

namespace kot {

// ---- optional launch profiler (events around kernel launches on the issuing stream) -----------------------
// PROF_CHAIN_F64: the FP64 GEMMs of the Schur matvec's eigen-row chain (counted apart from the other FP64
// GEMMs while g_prof_chain is set on the issuing thread).
enum ProfClass { PROF_GEMM_F64 = 0, PROF_EIG_ROUND = 1, PROF_GEMV_F64 = 2, PROF_GEMM_F32 = 3, PROF_GEMM_BF16 = 4,
                 PROF_POTENTIAL = 5, PROF_CHAIN_F64 = 6, PROF_NCLASS = 7 };
struct Profiler {
  bool on = false;
  struct Rec { int cls; double flops; double bytes; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  hipEvent_t get();
  // begin/end bracket one launch (or a fixed group of launches) of class cls
  void begin(hipStream_t st, int cls, double flops, double bytes);
  void end(hipStream_t st);
  void clear();
  ~Profiler();
};
extern thread_local Profiler* g_prof;
extern thread_local int g_prof_chain;

// ---- GEMM (FP64 MFMA): C = alpha * op(A) * diag(s) * op(B) + beta * C, row-major --------------------------
// Batched over grid.z with element strides sA, sB, sS, sC (0 for a shared operand).  lower != 0: only the
// 64x64 output tiles that meet the lower triangle (col <= row) are computed; entries above it are left
// unspecified, unless mirror != 0 (square symmetric results, m == n): then every strictly-lower tile also
// writes its transpose.  tri: known zero triangles of the operands, bit 1 op(A) upper, 2 op(A) lower,
// 4 op(B) upper, 8 op(B) lower; each tile then runs only over the K range where both can be nonzero.
// A single product with n == 1 and op(A) = A runs as a GEMV (HBM-bound, no matrix cores).
struct GemmArgs {
  int transa, transb, m, n, k;
  double alpha, beta;
  const double* A; int lda; long long sA;
  const double* s; long long sS;      // may be null
  const double* B; int ldb; long long sB;
  double* C; int ldc; long long sC;
  int batch;
  int lower, mirror, tri;
  // column-dot mode (D non-null, batch 1, no lower/mirror): instead of C, y_j = dalpha sum_i D_ij
  // (alpha op(A) diag(s) op(B))_ij + dbeta y_j, D m x n with leading dimension ldd; C is not touched
  const double* D = nullptr; int ldd = 0;
  double* y = nullptr; double dalpha = 1.0, dbeta = 0.0;
};
// y = a Q v + b K2 v + c v for square m x m row-major Q, K2 (K2 may be null; v, y device vectors)
hipError_t gemv2(int m, const double* Q, double a, const double* K2, double b, const double* v, double c, double* y,
                 hipStream_t st);
// Reserves the current device's pool of GEMM work lists (once per device and process; call outside any solve).
hipError_t gemm_reserve();
hipError_t gemm_f64(const GemmArgs& g, hipStream_t st);
// Same with an explicit launch shape: waves per workgroup (4, 8 or 16; 0 = default) and K splits (0 = from
// the split-K target of the size bucket).
hipError_t gemm_f64_cfg(const GemmArgs& g, hipStream_t st, int waves, int splits);
// Split-K workspace used by gemm_f64 on the calling thread (set per library call by the context; null or
// too small => no K split).
extern thread_local double* g_gemm_ws;
extern thread_local size_t g_gemm_ws_cap;  // doubles
// Split-K target workgroup count per size bucket (0 = never split); null => 512 everywhere.
constexpr int kTuneBuckets = 33;
inline int gemm_tune_bucket(int size) { const int b = (size + 127) / 128; return b < kTuneBuckets ? b : kTuneBuckets - 1; }
extern thread_local const int* g_gemm_tune;

// y[j] = alpha * sum_{r in [r0, r1)} A[r*lda + j] * B[r*ldb + j] + beta * y[j], j < n (column dots).
// part: workspace of at least kDiagParts * n doubles.
constexpr int kDiagParts = 16;
hipError_t diag_dot(int r0, int r1, int n, double alpha, const double* A, int lda, const double* B, int ldb,
                    double beta, double* y, double* part, hipStream_t st);

// ---- setup ------------------------------------------------------------------------------------------------
hipError_t gram_build(int l, int d, const double* xf, const double* yf, double sigma, double* Q, double* K,
                      hipStream_t st);
hipError_t mean_embedding(int n, int l, int d, const double* samples, const double* pts, double sigma,
                          double* w, hipStream_t st);
// sum_{i,j} k(x_i, x_j) / n^2 written to out[0] (d <= 64); part: workspace of mean_gram_part_size(n) doubles.
size_t mean_gram_part_size(int n);
hipError_t mean_gram(int n, int d, const double* x, double sigma, double* out, double* part, hipStream_t st);
hipError_t build_z(int l, int d, const double* xf, const double* yf, const double* wmu, const double* wnu,
                   double lam2, double* z, double* wsum, hipStream_t st);

// ---- Cholesky: R^T R = A + eps I (R upper). info[0] != 0 on a non-positive pivot. ----------------------------
// Linv (optional, l x l): receives X = L^-1 = R^-T (lower triangle, zeros above), computed beside the factor.
hipError_t cholesky_upper(int l, const double* A, double eps, double* R, double* work, int* info, hipStream_t st,
                          double* Linv = nullptr);

// ---- symmetric eigensolver (block Jacobi) ------------------------------------------------------------------
struct EigWork;
// Largest l of the allocation-free eigendecomposition (its scratch is a static device array).
constexpr int kNoAllocMaxL = 512;
size_t eigh_noalloc_scratch_bytes();
// Cold-start eigendecomposition of (Z + Z^T)/2 without allocating: full Jacobi sweeps in the static scratch
// array of `device` (which must be current); the scratch is shared by every call on that device.
hipError_t eigh_jacobi_noalloc(int device, int l, const double* Z, double* P, double* wv, int max_sweeps,
                               int inner_sweeps, double tol, int* sweeps, double* rel_off, hipStream_t st);
EigWork* eig_work_create(int lmax);
void eig_work_destroy(EigWork* w);
// Z (l x l) -> P (columns eigenvectors), wv ascending.  If P0 is non-null, starts from the basis P0
// (columns orthonormal).  Returns the sweep count through *sweeps, off/norm through *rel_off and the number
// of positive eigenvalues through *npos (may be null); the host has synchronized with the stream on return.
// tmp: workspace of tmp_mats >= 2 matrices of eig_mat_doubles(l) doubles each (blocked A and V); with a third
// (required for a warm start) a full sweep runs one launch per round instead of two, and with a fourth V is
// updated by two rounds at once.
size_t eig_mat_doubles(int l);
hipError_t eigh_jacobi(EigWork* w, int l, const double* Z, const double* P0, double* P, double* wv, double* tmp,
                       int tmp_mats, int max_sweeps, int inner_sweeps, double tol, int* sweeps, double* rel_off,
                       int* npos, hipStream_t st);

// ---- vector kernels -----------------------------------------------------------------------------------------
hipError_t vec_fill(int n, double v, double* x, hipStream_t st);
hipError_t mat_fill(int rows, int cols, double v, double* C, int ldc, hipStream_t st);
hipError_t vec_copy(int n, const double* x, double* y, hipStream_t st);
// y = a*x + b*y
hipError_t vec_axpby(int n, double a, const double* x, double b, double* y, hipStream_t st);
// z = a*x + b*y
hipError_t vec_lincomb(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t st);
// X += a * I  (l x l)
hipError_t add_diag(int l, double a, double* X, hipStream_t st);
// Diagonal kernel factor (the sparsity of Remark 4.5): out[0..1] = max off-diagonal and max diagonal |A_ij|;
// R = diag(sqrt(K_ii)) as a dense matrix with rd its diagonal and Linv = R^-T (optional), info = 0 or the first
// non-positive K_ii (1-based); out = diag(rd^power g) for power +-2; y = alpha diag(rd^2) diag(X) + beta y;
// B = P^T diag(rd).
hipError_t offdiag_absmax(int l, const double* A, double* out, hipStream_t st);
hipError_t diag_factor(int l, const double* K, double* R, double* rd, double* Linv, int* info, hipStream_t st);
hipError_t diag_gram(int l, const double* rd, int power, const double* g, double* out, hipStream_t st);
hipError_t phi_diag(int l, const double* rd, const double* X, double alpha, double beta, double* y, hipStream_t st);
hipError_t transpose_scale(int l, const double* P, const double* rd, double* B, hipStream_t st);
// Z = 0.5 * (Z + Z^T)
hipError_t symmetrize(int l, double* Z, hipStream_t st);
// Deterministic reductions: out[0] = sum x*y; partials in part (>= 2 kRedBlocks doubles).  dot2 forms one or
// two dot products (x2 null: one) in the same launches.
constexpr int kRedBlocks = 256;
hipError_t dot(int n, const double* x, const double* y, double* out, double* part, hipStream_t st);
// out = X - Y (n entries) with the block partials of |out|^2 into part; returns the number of partials (< 0 on a
// launch error).  resid_norms_final: o1 = |r1|^2 (length l), o2 = the partials' sum (one workgroup).
int mat_sub_sq(long long n, const double* X, const double* Y, double* out, double* part, hipStream_t st);
hipError_t resid_norms_final(int nb, const double* part, int l, const double* r1, double* o1, double* o2,
                             hipStream_t st);
hipError_t dot2(long long n, const double* x1, const double* y1, double* o1, const double* x2, const double* y2,
                double* o2, double* part, hipStream_t st);
// Z = (M + M^T)/2 + c I with M = X - a T (l x l; Z must not alias X or T)
hipError_t form_z(int l, const double* X, double a, const double* T, double c, double* Z, hipStream_t st);
// CG update with a device step length: alpha = rr / pAp[0] (0 when pAp[0] <= 0); x += alpha p; r -= alpha Ap.
// Conjugate gradients with the scalars on the device (n <= 8192, one workgroup per call).  st holds r.r, x.x,
// a stop flag and the iteration count (indices below).  cg_init: x = 0, r = p = b and the test at the start;
// cg_tail: the vector part of one iteration given Ap (Ap + addmu p is the operator's product), a no-op once
// stopped.  Stop: |r| <= tau min(1, kr |x|) (or |r| <= fixed when fixed > 0), cap iterations, or p.Ap <= 0.
// dinv (n, may be null): the inverse of a diagonal preconditioner (preconditioned CG; the test stays on r).
constexpr int kCgRR = 0, kCgXX = 1, kCgDone = 2, kCgIt = 3, kCgRZ = 4;
hipError_t cg_init(int n, const double* b, double* x, double* r, double* p, double* st, double tau, double kr,
                   double fixed, int cap, hipStream_t s, const double* dinv = nullptr);
hipError_t cg_tail(int n, double* st, double* p, const double* Ap, double addmu, double* x, double* r, double tau,
                   double kr, double fixed, int cap, hipStream_t s, const double* dinv = nullptr);
// Symmetric QMR with the scalars on the device (same st layout, tests and limits as CG; st also holds tau and
// theta).  sqmr_init: x = d = e = 0, r = s = b, q = D^-1 b; sqmr_tail: one iteration given t = A q.  s is the
// true residual b - A x; the stopping test runs on it.
hipError_t sqmr_init(int n, const double* b, double* x, double* r, double* q, double* d, double* e, double* s,
                     double* st, double tau, double kr, double fixed, int cap, hipStream_t s_, const double* dinv);
hipError_t sqmr_tail(int n, double* st, double* q, const double* t, double* x, double* r, double* d, double* e,
                     double* s, double tau, double kr, double fixed, int cap, hipStream_t s_, const double* dinv);
// d_i = cq Q_ii + mu + ckk KK_ii (KK may be null); out_i = 1 / d_i
hipError_t schur_diag_base(int l, const double* Q, double cq, double mu, const double* KK, double ckk, double* d,
                           hipStream_t st);
hipError_t vec_recip(int n, const double* d, double* out, hipStream_t st);
hipError_t cg_step(int n, double rr, const double* pAp, const double* p, const double* Ap, double* x, double* r,
                   hipStream_t st);
// out[0] = max_i sum_j |A_ij| (row-sum norm)
hipError_t rowsum_abs_max(int l, const double* A, bool square_entries, double* out, double* part, hipStream_t st);
// out_int[0] = number of nonzero entries strictly below the diagonal of R (l x l)
hipError_t count_lower_nonzero(int l, const double* R, int* out_int, hipStream_t st);
// count of w[i] > 0 (ascending w): out_int[0]
hipError_t count_positive(int l, const double* w, int* out_int, hipStream_t st);
// Psi rows for the eigen-index range [r0, r0 + m): H[r][j] = weight(r, j) * C[r][j] (in place), with
// weight per Section 4.3; 'complement' selects the complement form used when |alpha| > l/2; 'half_diag'
// scales the within-set block by 1/2 (for G + G^T) and 'double_off' doubles the cross block (CG chain).
hipError_t psi_hadamard(int l, int a, int r0, int m, double mu, const double* w, double* C, int ldc,
                        bool complement, double diag_scale, double off_scale, hipStream_t st);
// out = P_S diag(w_S) P_S^T restricted to eigen-index set S = [r0, r0+m): via gemm (helper in host code)
// X_out = X - Y ; also norm
hipError_t mat_sub(int n, const double* X, const double* Y, double* out, hipStream_t st);
hipError_t transpose(int l, const double* A, double* At, hipStream_t st);
hipError_t hadamard_square(int n, const double* A, double* out, hipStream_t st);
// G + G^T into out (l x l): out[i][j] = a*(G[i][j] + G[j][i]) + b*S[i][j]
hipError_t sym_plus(int l, const double* G, double a, const double* S, double b, double* out, hipStream_t st);
// scale columns: out[i][j] = A[i][j] * s[j]
hipError_t scale_cols(int rows, int cols, const double* A, int lda, const double* s, double* out, int ldo,
                      hipStream_t st);

// ---- warm-start network (k_mlp.hip) ----------------------------------------------------------------------
constexpr int kFeatures = 12;
struct GemmF32Args {
  int ta, tb, m, n, k;
  const float* A; int lda;
  const float* B; int ldb;
  float* C; int ldc;
  float beta;
  const float* bias;   // per output column, may be null
  int act;             // 1 = relu
  const float* mask;   // multiply by (mask > 0), may be null
  int ldm;
};
hipError_t gemm_f32(const GemmF32Args& g, hipStream_t st);
hipError_t colsum_f32(int rows, int cols, const float* X, float* out, float* part, hipStream_t st);
hipError_t mse_grad(int n, const float* out, const float* y, float* dout, double* loss, double* part, hipStream_t st);
hipError_t adam_f32(int n, float* th, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, int t,
                    hipStream_t st);
// X (l x kFeatures, FP32); rs: workspace 3l doubles; pooled: 2 device doubles
hipError_t features(int l, const double* Q, const double* z, const double* wsum, const double* K, const double* KK,
                    double lam1, double* rs, double* pooled, float* X, hipStream_t st);
hipError_t f32_to_f64_scaled(int n, const float* x, double s, double* y, hipStream_t st);
// Y = R^{-1} (R upper triangular, l x l); T: l x l workspace.
hipError_t trtri_upper(int l, const double* R, double* Y, double* T, hipStream_t st);
// d = ((Q g - z)/(2 lam2)) on predicted-active points (g_i <= -0.9 lambda1), zeroed below frac * mean of the
// positive entries; part: >= 128 doubles.
hipError_t closed_start(int l, const double* Q, const double* z, double lam1, double* g, hipStream_t st);
hipError_t lift_diag(int l, const double* Qg, const double* z, const double* g, double lam1, double lam2, double frac,
                     double* d, double* part, hipStream_t st);

// ---- potentials and transport map (k_pot.hip) ----------------------------------------------------------------
// u(q_i) = (w(q_i) - sum_j gamma_j k(fill_j, q_i)) / (2 lam2) and, when T is non-null, T(q_i) = q_i - grad u(q_i),
// for m query rows q (m x d, d <= 64), samples (ns x d), fill (l x d).  part: potential_part_size(m, d, splits)
// doubles; splits from potential_splits.
int potential_dim(int d);
size_t potential_part_size(int m, int d, int splits);
int potential_splits(int m, int ns, int l);
hipError_t potential_eval(int m, int d, const double* q, const double* samples, int ns, const double* fill, int l,
                          const double* gamma, double sigma, double lam2, int splits, double* part, double* u,
                          double* T, hipStream_t st);

// ---- reduced-precision CG chain (k_lowp.hip) --------------------------------------------------------------
struct LowpArgs {
  int m, n, k;
  const float* A; int lda;   // m x k, row-major
  const double* s;           // diag scale on k (may be null)
  const float* B; int ldb;   // n x k (transb) or k x n
  int transb;
  float* C; int ldc;
  // Psi epilogue (see psi_hadamard): row r of C is eigen-index r0 + r
  int l, a, r0;
  double mu;
  const double* w;
  int complement;
  double diag_scale, off_scale;
};
// mode: 0 FP32 products, 1 BF16, 2 split BF16 (three products); FP32 accumulation
hipError_t gemm_lowp(const LowpArgs& g, int mode, bool psi, hipStream_t st);
hipError_t f64_to_f32(long long n, const double* x, float* y, hipStream_t st);
// BF16 chain of the Schur matvec (gfx950 MFMA, see k_lowp.hip): operands rounded once per Newton direction.
struct ChainArgs {
  int m, l, ldp, r0;                       // chain rows, size, padded leading dimension, first eigen-row
  const double* v;                         // matvec input (length l)
  const unsigned short *Bh, *BhT, *Bl, *BlT;  // bf16 B and B^T (hi, lo), ldp x ldp, zero padded
  unsigned short *Hh, *Hl;                 // bf16 H (hi, lo), m x ldp
  // Psi epilogue (see psi_hadamard)
  int a;
  double mu;
  const double* w;
  int complement;
  double diag_scale, off_scale;
  // column-dot epilogue: y[j] += alpha sum_r D[r][j] (H B)[r][j]
  const float* D; int ldd;
  double alpha;
  double* part;                            // >= ceil(m / 32) * l doubles
  double* y;
};
int chain_ldp(int l);
hipError_t chain_prep(int l, int ldp, const double* B, unsigned short* Bh, unsigned short* BhT, unsigned short* Bl,
                      unsigned short* BlT, hipStream_t st);
hipError_t chain_bf16(const ChainArgs& g, bool split, hipStream_t st);
// y[j] += alpha * sum_{r < m} A[r][j] B[r][j]; part >= 16 n doubles
hipError_t diag_dot_lowp(int m, int n, double alpha, const float* A, int lda, const float* B, int ldb, double* y,
                         double* part, hipStream_t st);

}  // namespace kot

#define KOT_HIP_TRY(expr)                                   \
  do {                                                      \
    hipError_t _e = (expr);                                 \
    if (_e != hipSuccess) return _e;                        \
  } while (0)
