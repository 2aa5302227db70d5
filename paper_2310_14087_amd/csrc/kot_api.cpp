// C-ABI of libkotssn and the host orchestration of the SSN method (Algorithms 1 and 2).
// Every arithmetic step runs in the HIP kernels of this library; the host only sequences launches and reads
// back the scalars that the algorithm branches on (norms, inner products, the eigenvalue count).
#include "kotssn.h"
#include "kot_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <functional>
#include <mutex>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

using namespace kot;

namespace {

constexpr int kScalarDoubles = 64, kScalarInts = 16;
constexpr size_t kScalarBytes = kScalarDoubles * sizeof(double) + kScalarInts * sizeof(int);
// scalar slots: 0-3 per-call temporaries; residual norms (|r1|^2, |r2|^2) of the EG point 4-5 and of the trial
// 6-7; the theta-rule dots 8-11; inputs of the default EG step 12-13; |z|^2 14; refinement scalars 16-19;
// the largest off-diagonal and diagonal entries of K + eps I 20-21;
// pooled feature statistics 24-25; the device-resident CG / QMR state 32-38
enum : int { SL_TMP = 0, SL_R1 = 2, SL_VN = 4, SL_TN = 6, SL_THETA = 8, SL_ETA = 12, SL_ZZ = 14, SL_RR = 16, SL_PAP = 17,
             SL_XX = 18, SL_KD = 20, SL_POOL = 24, SL_CG = 32 };

struct State {  // an iterate w = (gamma, X) with its residual and the spectral data of Z
  double* g = nullptr;
  double* X = nullptr;
  double* r1 = nullptr;
  double* r2 = nullptr;
  double* P = nullptr;
  double* s = nullptr;
  int a = 0;
  double r1n = 0.0, r2n = 0.0, rn = 0.0;
  bool has_eig = false;
};

struct CoreView {  // dual data of Eq. (3.4) on the device
  int l = 0;
  const double* Q = nullptr;
  const double* z = nullptr;
  const double* R = nullptr;
  const double* wsum = nullptr;
  double q2 = 0.0;
  double lam1 = 0.0, lam2 = 0.0;
  double* KK = nullptr;  // (R^T R) o (R^T R)
  const double* Linv = nullptr;  // R^-T when the factorization produced it (else the lift inverts R itself)
  const double* rd = nullptr;    // non-null: R is diagonal (kdiag_tol), rd its diagonal; products with R scale
  int kb_state = 0;      // the context's K buffer: 0 unrelated, 1 holds R^T R = K + eps I, 2 and KK is formed
};

struct Prelude {  // setup results computed on the second stream while the factorization runs
  double q2 = 0.0, eta = 0.0, zz = 0.0;
};

struct SideRunner;

}  // namespace

struct kot_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  EigWork* eig = nullptr;
  int cap = 0;  // workspace l capacity
  std::vector<void*> bufs;
  // scalar exchange: kScalarDoubles doubles then kScalarInts ints, device and pinned host, copied whole by
  // every sync_read (slots below)
  double* dsc = nullptr;
  double* hsc = nullptr;      // pinned, mapped and coherent: written by a device copy, read by the host
  double* hsc_dev = nullptr;  // device address of hsc
  int* dint = nullptr;
  int* hint = nullptr;
  double* part = nullptr;      // reduction partials (>= max(kRedBlocks, kDiagParts*l, n, q^2 tile pairs))
  size_t part_cap = 0;
  double* gemm_ws = nullptr;   // split-K partial tiles (16 l^2 doubles: up to 16 K slices of an l x l product)
  size_t gemm_ws_cap = 0;
  // matrices (cap x cap)
  double *Qb, *Rb, *Kb, *KKb, *Z, *T1, *T2, *T3, *T4, *Bm, *dX, *Mr, *eigtmp, *Pe1, *Pe2, *Xh;
  // vectors (cap)
  double *zb, *wsumb, *wmu, *wnu, *dg, *a1, *cx, *cr, *cp, *cAp, *cdinv, *rdb, *qd, *qe, *qs, *vtmp, *gh, *s_e1, *s_e2, *r1h, *lx, *lr, *lp, *lAp;
  float *Bf = nullptr, *Cf = nullptr, *Ef = nullptr;  // reduced-precision chain operands
  // BF16 chain: bfloat16 B, B^T (hi and lo) and H (hi and lo), each ldp x ldp (ldp = chain_ldp(cap))
  unsigned short *Bh = nullptr, *BhT = nullptr, *Bl = nullptr, *BlT = nullptr, *Hh = nullptr, *Hl = nullptr;
  State S[4];  // 0: w, 1: trial, 2: v, 3: scratch
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  Profiler prof;
  // warm-start network workspace
  std::vector<void*> mbufs;
  size_t mlp_rows = 0, mlp_h = 0;
  float *fA1 = nullptr, *fA2 = nullptr, *fdZ1 = nullptr, *fdZ2 = nullptr, *fout = nullptr, *fdout = nullptr,
        *fpart = nullptr, *fX = nullptr;
  double* rs3 = nullptr;
  // batched solves: child contexts (own stream and workspace), one host worker thread each
  std::vector<kot_ctx*> lanes;
  // potentials: split partial sums (grown on demand)
  double* pot_part = nullptr;
  size_t pot_part_cap = 0;
  // split-K targets per size bucket (autotuner)
  int tune[kTuneBuckets];
  bool tuned = false;
  // second and third streams, each with a host thread, for the extragradient branch of Algorithm 2 (created on
  // first use)
  SideRunner* side = nullptr;
  SideRunner* side2 = nullptr;  // the extragradient step's second projection
  // the triangular inverse of the lift as one graph (about thirty small launches), per (l, buffers)
  hipGraphExec_t trtri_graph = nullptr;
  int trtri_l = 0;
  const void* trtri_key[4] = {nullptr, nullptr, nullptr, nullptr};
  bool trtri_graph_failed = false;
  bool is_lane = false;  // a child context of kot_solve_batched
};

namespace {

kot_status fail(kot_ctx* c, kot_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return st;
}

#define HIPCHK(expr)                                                                        \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(ctx, KOT_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(_e), \
                  __FILE__, __LINE__);                                                      \
  } while (0)

#define KCHK(expr)                  \
  do {                              \
    kot_status _s = (expr);         \
    if (_s < 0) return _s;          \
  } while (0)

void free_ws(kot_ctx* c) {
  for (void* p : c->bufs) hipFree(p);
  c->bufs.clear();
  c->gemm_ws = nullptr;
  c->gemm_ws_cap = 0;
  g_gemm_ws = nullptr;
  g_gemm_ws_cap = 0;
  if (c->eig) { eig_work_destroy(c->eig); c->eig = nullptr; }
  c->cap = 0;
}

kot_status ensure_ws(kot_ctx* ctx, int l, int nmax) {
  HIPCHK(hipSetDevice(ctx->device));
  const size_t need_part = std::max<size_t>({(size_t)2 * kRedBlocks, (size_t)kDiagParts * l + 64, (size_t)nmax + 64,
                                             (size_t)l + 64, nmax > 0 ? mean_gram_part_size(nmax) : (size_t)0,
                                             (size_t)((l + 31) / 32) * l + 64});  // BF16 chain column dots
  if (l <= ctx->cap && need_part <= ctx->part_cap) return KOT_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  free_ws(ctx);
  const int cap = std::max(l, ctx->cap);
  const size_t mm = (size_t)cap * cap * sizeof(double);
  const size_t vv = (size_t)cap * sizeof(double);
  auto alloc = [&](size_t bytes) -> double* {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    ctx->bufs.push_back(p);
    return (double*)p;
  };
  double** mats[] = {&ctx->Qb, &ctx->Rb, &ctx->Kb, &ctx->KKb, &ctx->Z, &ctx->T1, &ctx->T2, &ctx->T3, &ctx->T4,
                     &ctx->Bm, &ctx->dX, &ctx->Mr, &ctx->Pe1, &ctx->Pe2, &ctx->Xh};
  for (double** m : mats)
    if (!(*m = alloc(mm))) return fail(ctx, KOT_ERR_OOM, "workspace allocation failed (l=%d)", cap);
  // the eigensolver's blocked A, V, second A and second V (each over the block-padded size)
  if (!(ctx->eigtmp = alloc(4 * eig_mat_doubles(cap) * sizeof(double))))
    return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  double** vecs[] = {&ctx->zb, &ctx->wsumb, &ctx->wmu, &ctx->wnu, &ctx->dg, &ctx->a1, &ctx->cx, &ctx->cr, &ctx->cp,
                     &ctx->cAp, &ctx->cdinv, &ctx->rdb, &ctx->qd, &ctx->qe, &ctx->qs, &ctx->vtmp, &ctx->gh, &ctx->s_e1, &ctx->s_e2, &ctx->r1h, &ctx->lx, &ctx->lr, &ctx->lp,
                     &ctx->lAp};
  for (double** v : vecs)
    if (!(*v = alloc(vv))) return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  for (auto& s : ctx->S) {
    if (!(s.g = alloc(vv)) || !(s.X = alloc(mm)) || !(s.r1 = alloc(vv)) || !(s.r2 = alloc(mm)) ||
        !(s.P = alloc(mm)) || !(s.s = alloc(vv)))
      return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
    s.has_eig = false;
  }
  if (!(ctx->part = alloc(need_part * sizeof(double)))) return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  ctx->part_cap = need_part;
  if (!(ctx->gemm_ws = alloc(16 * mm))) return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  if (!(ctx->Bf = (float*)alloc(mm / 2)) || !(ctx->Cf = (float*)alloc(mm / 2)) || !(ctx->Ef = (float*)alloc(mm / 2)))
    return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  {
    const size_t lp = (size_t)chain_ldp(cap), hb = lp * lp * sizeof(unsigned short);
    unsigned short** hbufs[] = {&ctx->Bh, &ctx->BhT, &ctx->Bl, &ctx->BlT, &ctx->Hh, &ctx->Hl};
    for (unsigned short** b : hbufs)
      if (!(*b = (unsigned short*)alloc(hb))) return fail(ctx, KOT_ERR_OOM, "workspace allocation failed");
  }
  ctx->gemm_ws_cap = 16 * (size_t)cap * cap;
  g_gemm_ws = ctx->gemm_ws;
  g_gemm_ws_cap = ctx->gemm_ws_cap;
  ctx->eig = eig_work_create(cap);
  if (!ctx->eig) return fail(ctx, KOT_ERR_OOM, "eigensolver workspace allocation failed");
  ctx->cap = cap;
  return KOT_OK;
}

// Copies every scalar slot to the host and waits for the stream: each host value read afterwards is that of
// the last kernel enqueued before this call that wrote its slot.
kot_status sync_read(kot_ctx* ctx, int = 0, int = 0) {
  static_assert(kScalarBytes % 16 == 0, "scalar block copied as double pairs");
  HIPCHK(vec_copy((int)(kScalarBytes / sizeof(double)), ctx->dsc, ctx->hsc_dev, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

// ---- GEMM helpers ------------------------------------------------------------------------------------------
// tri: known zero triangles of op(A) / op(B) (GemmArgs::tri); sym: the result is symmetric (m == n, and C
// symmetric when beta != 0), so only the lower tiles are computed and mirrored.
hipError_t mm(hipStream_t st, int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda,
              const double* s, const double* B, int ldb, double beta, double* C, int ldc, int tri = 0,
              bool sym = false) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (k <= 0) {
    if (beta != 0.0) return hipErrorInvalidValue;  // not needed by callers
    return mat_fill(m, n, 0.0, C, ldc, st);
  }
  GemmArgs g{};
  g.transa = ta; g.transb = tb; g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = beta;
  g.A = A; g.lda = lda; g.s = s; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc; g.batch = 1;
  g.tri = tri;
  if (sym && m == n) { g.lower = 1; g.mirror = 1; }
  return gemm_f64(g, st);
}

constexpr int TRI_A_UPPER = 1, TRI_A_LOWER = 2, TRI_B_UPPER = 4, TRI_B_LOWER = 8;

// y_j = dalpha sum_i D_ij (alpha op(A) diag(s) op(B))_ij + dbeta y_j, the product never written out (its column
// dots against D are taken in the GEMM's epilogue).  D is m x n with leading dimension ldd.
hipError_t mm_coldot(hipStream_t st, int ta, int tb, int m, int n, int k, double alpha, const double* A, int lda,
                     const double* s, const double* B, int ldb, int tri, const double* D, int ldd, double dalpha,
                     double dbeta, double* y) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (k <= 0) return hipErrorInvalidValue;
  GemmArgs g{};
  g.transa = ta; g.transb = tb; g.m = m; g.n = n; g.k = k; g.alpha = alpha; g.beta = 0.0;
  g.A = A; g.lda = lda; g.s = s; g.B = B; g.ldb = ldb; g.C = nullptr; g.ldc = n; g.batch = 1;
  g.tri = tri;
  g.D = D; g.ldd = ldd; g.y = y; g.dalpha = dalpha; g.dbeta = dbeta;
  return gemm_f64(g, st);
}

// out = Phi*(g) = R diag(g) R^T  (R upper: the k-th term touches only rows and columns <= k)
kot_status phi_star(kot_ctx* ctx, const CoreView& cv, const double* g, double* out) {
  const int l = cv.l;
  if (cv.rd) {
    HIPCHK(diag_gram(l, cv.rd, 2, g, out, ctx->stream));
    return KOT_OK;
  }
  HIPCHK(mm(ctx->stream, 0, 1, l, l, l, 1.0, cv.R, l, g, cv.R, l, 0.0, out, l, TRI_A_UPPER | TRI_B_LOWER, true));
  return KOT_OK;
}

// y = alpha*Phi(X) + beta*y, Phi(X)_i = R[:,i]^T X R[:,i] = sum_r R_ri (X R)_ri (X R never written out)
kot_status phi_op(kot_ctx* ctx, const CoreView& cv, const double* X, double alpha, double beta, double* y) {
  const int l = cv.l;
  if (cv.rd) {
    HIPCHK(phi_diag(l, cv.rd, X, alpha, beta, y, ctx->stream));
    return KOT_OK;
  }
  HIPCHK(mm_coldot(ctx->stream, 0, 0, l, l, l, 1.0, X, l, nullptr, cv.R, l, TRI_B_UPPER, cv.R, l, alpha, beta, y));
  return KOT_OK;
}

// r1 = (Q g - z)/(2 lam2) - Phi(X)
kot_status r1_op(kot_ctx* ctx, const CoreView& cv, const double* g, const double* X, double* r1) {
  const int l = cv.l;
  // r1 = Q g  (as an l x 1 product)
  HIPCHK(mm(ctx->stream, 0, 0, l, 1, l, 1.0, cv.Q, l, nullptr, g, 1, 0.0, r1, 1));
  HIPCHK(vec_axpby(l, -1.0 / (2.0 * cv.lam2), cv.z, 1.0 / (2.0 * cv.lam2), r1, ctx->stream));
  KCHK(phi_op(ctx, cv, X, -1.0, 1.0, r1));
  return KOT_OK;
}

// Eigendecomposition of Z (warm basis P0 or null); *npos receives the number of positive eigenvalues.  The
// host is synchronized with the stream on return.
kot_status eig_run(kot_ctx* ctx, int l, const double* Z, const double* P0, double* P, double* w, const kot_params* p,
                   int* sweeps_acc, int* npos) {
  int sw = 0;
  double rel = 0.0;
  const int max_sw = p->eig_max_sweeps > 0 ? p->eig_max_sweeps : 30;
  const int inner = p->eig_inner_sweeps > 0 ? p->eig_inner_sweeps : 1;
  HIPCHK(eigh_jacobi(ctx->eig, l, Z, P0, P, w, ctx->eigtmp, 4, max_sw, inner, 1e-14, &sw, &rel, npos, ctx->stream));
  if (sweeps_acc) *sweeps_acc += sw;
  if (!(rel <= 1e-14)) {
    if (!std::isfinite(rel)) return fail(ctx, KOT_ERR_NUMERIC, "non-finite matrix in eigensolver");
    return fail(ctx, KOT_ERR_EIG, "Jacobi did not converge in %d sweeps (off/norm = %.3e)", sw, rel);
  }
  return KOT_OK;
}

// Pi(Z) = P_alpha diag(w_alpha) P_alpha^T given ascending spectral data with a positives; when more than half
// the eigenvalues are positive, the same matrix as Z - P_abar diag(w_abar) P_abar^T (inner size l - a).
kot_status proj_from_eig(kot_ctx* ctx, int l, const double* Z, const double* P, const double* w, int a, double* out) {
  if (a <= l - a) {
    HIPCHK(mm(ctx->stream, 0, 1, l, l, a, 1.0, P + (l - a), l, w + (l - a), P + (l - a), l, 0.0, out, l, 0, true));
  } else {
    HIPCHK(vec_copy(l * l, Z, out, ctx->stream));
    if (l - a > 0) HIPCHK(mm(ctx->stream, 0, 1, l, l, l - a, -1.0, P, l, w, P, l, 1.0, out, l, 0, true));
  }
  return KOT_OK;
}

// Residual map Eq. (4.2) at state s (g, X set); fills r1, r2, P, s, a.  P0: warm basis or null.  The squared
// norms go to slots (slot, slot + 1); with defer the host reads them later (finish_norms after a sync_read),
// otherwise at once.
void finish_norms(kot_ctx* ctx, State& s, int slot) {
  s.r1n = std::sqrt(ctx->hsc[slot]);
  s.r2n = std::sqrt(ctx->hsc[slot + 1]);
  s.rn = s.r1n + s.r2n;
}

kot_status residual_state(kot_ctx* ctx, const CoreView& cv, State& s, const double* P0, const kot_params* p,
                          int* sweeps_acc, int slot = SL_TMP, bool defer = false) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  KCHK(phi_star(ctx, cv, s.g, ctx->T1));
  HIPCHK(form_z(l, s.X, 1.0, ctx->T1, -cv.lam1, ctx->Z, st));
  KCHK(eig_run(ctx, l, ctx->Z, P0, s.P, s.s, p, sweeps_acc, &s.a));
  KCHK(proj_from_eig(ctx, l, ctx->Z, s.P, s.s, s.a, ctx->T1));
  // r2 = X - Pi(Z) with its squared norm's partials in the same pass; |r1|^2 and |r2|^2 land in (slot, slot + 1)
  const int nb = mat_sub_sq((long long)l * l, s.X, ctx->T1, s.r2, ctx->part, st);
  if (nb < 0) return fail(ctx, KOT_ERR_HIP, "mat_sub_sq: launch failed");
  KCHK(r1_op(ctx, cv, s.g, s.X, s.r1));
  HIPCHK(resid_norms_final(nb, ctx->part, l, s.r1, ctx->dsc + slot, ctx->dsc + slot + 1, st));
  s.has_eig = true;
  if (!defer) {
    KCHK(sync_read(ctx));
    finish_norms(ctx, s, slot);
  }
  return KOT_OK;
}

// r1 of state s and its squared norm in the SL_VN slot of ctx's scalars; with sync, read back at once.
kot_status r1_only(kot_ctx* ctx, const CoreView& cv, State& s, bool sync = true) {
  KCHK(r1_op(ctx, cv, s.g, s.X, s.r1));
  HIPCHK(dot(cv.l, s.r1, s.r1, ctx->dsc + SL_VN, ctx->part, ctx->stream));
  if (sync) KCHK(sync_read(ctx));
  return KOT_OK;
}

// ---- operator T (Section 4.3) via the G + G^T decomposition -----------------------------------------------
struct TPlan {
  int l, a;
  bool comp;   // complement form (|alpha| > l/2)
  int r0, m;   // eigen-index set of the rows used: alpha, or alpha-bar in the complement form
  double mu;
  const double* P;
  const double* w;
};

TPlan make_tplan(int l, int a, double mu, const double* P, const double* w) {
  TPlan t;
  t.l = l; t.a = a; t.mu = mu; t.P = P; t.w = w;
  t.comp = (a > l - a);
  if (!t.comp) { t.r0 = l - a; t.m = a; }
  else { t.r0 = 0; t.m = l - a; }
  return t;
}

// out = T[S]; uses T3, T4 (and out must differ from S and from T3/T4)
kot_status t_apply(kot_ctx* ctx, const TPlan& tp, const double* S, double* out) {
  const int l = tp.l;
  hipStream_t st = ctx->stream;
  if (tp.m == 0) {
    if (!tp.comp) HIPCHK(vec_fill(l * l, 0.0, out, st));               // alpha empty: T = 0
    else HIPCHK(vec_lincomb(l * l, 1.0 / tp.mu, S, 0.0, S, out, st));  // alpha-bar empty: T = S/mu
    return KOT_OK;
  }
  double* U = ctx->T3;   // m x l
  double* Y = ctx->T4;   // m x l
  // U = P_set^T S
  HIPCHK(mm(st, 1, 0, tp.m, l, l, 1.0, tp.P + tp.r0, l, nullptr, S, l, 0.0, U, l));
  // Y = U P  (= P_set^T S P)
  HIPCHK(mm(st, 0, 0, tp.m, l, l, 1.0, U, l, nullptr, tp.P, l, 0.0, Y, l));
  // Y <- W (weights with 1/2 on the within-set block)
  HIPCHK(psi_hadamard(l, tp.a, tp.r0, tp.m, tp.mu, tp.w, Y, l, tp.comp, 0.5, 1.0, st));
  // U = W P^T
  HIPCHK(mm(st, 0, 1, tp.m, l, l, 1.0, Y, l, nullptr, tp.P, l, 0.0, U, l));
  // G = P_set U   (l x l) into Y? Y is only m x l sized conceptually but buffers are l x l
  HIPCHK(mm(st, 0, 0, l, l, tp.m, 1.0, tp.P + tp.r0, l, nullptr, U, l, 0.0, Y, l));
  if (!tp.comp) HIPCHK(sym_plus(l, Y, 1.0, nullptr, 0.0, out, st));
  else HIPCHK(sym_plus(l, Y, -1.0, S, 1.0 / tp.mu, out, st));
  return KOT_OK;
}

// y = (Q/(2 lam2) + mu I + Phi T Phi*) v  with the B = P^T R chain (Bm holds B)
kot_status schur_matvec(kot_ctx* ctx, const CoreView& cv, const TPlan& tp, const double* v, double* y) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  // y = Q v / (2 lam2) + mu v (+ (1/mu) (K o K) v in the complement form), one pass
  HIPCHK(gemv2(l, cv.Q, 1.0 / (2.0 * cv.lam2), tp.comp ? cv.KK : nullptr, 1.0 / tp.mu, v, tp.mu, y, st));
  if (tp.m == 0) return KOT_OK;
  const double* Bs = ctx->Bm + (long long)tp.r0 * l;
  double* C = ctx->T3;
  struct ChainTag {  // the profiler counts the chain's products in their own class
    ChainTag() { g_prof_chain = 1; }
    ~ChainTag() { g_prof_chain = 0; }
  } tag;
  // C = B_set diag(v) B^T   (m x l)
  HIPCHK(mm(st, 0, 1, tp.m, l, l, 1.0, Bs, l, v, ctx->Bm, l, 0.0, C, l));
  // H = [Psi o C] with the cross block doubled
  HIPCHK(psi_hadamard(l, tp.a, tp.r0, tp.m, tp.mu, tp.w, C, l, tp.comp, 1.0, 2.0, st));
  // y_i += (+/-) sum_{r in set} B_ri E_ri with E = H B (E's column dots taken in the product's epilogue)
  HIPCHK(mm_coldot(st, 0, 0, tp.m, l, l, 1.0, C, l, nullptr, ctx->Bm, l, 0, Bs, l, tp.comp ? -1.0 : 1.0, 1.0, y));
  return KOT_OK;
}

// Jacobi (diagonal) preconditioner of the Schur system (an addition; the paper runs plain CG): the diagonal
// of M = Q/(2 lam2) + mu I + Phi T Phi* is M_ii = Q_ii/(2 lam2) + mu + [(B o B)^T Psi (B o B)]_ii (B = P^T R),
// formed with the matvec's eigen-row chain: E = H (B o B), H the chain's Psi weights (cross block doubled),
// then +/- sum over the chain's rows r of (B o B)_ri E_ri, and (1/mu) (K o K)_ii in the complement form.
// dinv receives 1 / M_ii.  Uses T1 and T3.
kot_status schur_dinv(kot_ctx* ctx, const CoreView& cv, const TPlan& tp, double* dinv) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  HIPCHK(schur_diag_base(l, cv.Q, 1.0 / (2.0 * cv.lam2), tp.mu, tp.comp ? cv.KK : nullptr, 1.0 / tp.mu, dinv, st));
  if (tp.m > 0) {
    double* D2 = ctx->T1;
    double* H = ctx->T3;
    HIPCHK(hadamard_square(l * l, ctx->Bm, D2, st));
    HIPCHK(mat_fill(tp.m, l, 1.0, H, l, st));
    HIPCHK(psi_hadamard(l, tp.a, tp.r0, tp.m, tp.mu, tp.w, H, l, tp.comp, 1.0, 2.0, st));
    HIPCHK(mm_coldot(st, 0, 0, tp.m, l, l, 1.0, H, l, nullptr, D2, l, 0, D2 + (long long)tp.r0 * l, l,
                     tp.comp ? -1.0 : 1.0, 1.0, dinv));
  }
  HIPCHK(vec_recip(l, dinv, dinv, st));
  return KOT_OK;
}

// Same operator with the chain in reduced precision (Bf holds B in FP32): FP32/BF16 products, FP32
// accumulation, FP64 for the Q and (K o K) terms.
kot_status schur_matvec_lowp(kot_ctx* ctx, const CoreView& cv, const TPlan& tp, const double* v, double* y, int mode) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  // y = Q v / (2 lam2) + mu v (+ (1/mu) (K o K) v in the complement form), FP64, one pass
  HIPCHK(gemv2(l, cv.Q, 1.0 / (2.0 * cv.lam2), tp.comp ? cv.KK : nullptr, 1.0 / tp.mu, v, tp.mu, y, st));
  if (tp.m == 0) return KOT_OK;
  if (mode != 0) {  // BF16 or split BF16 on the gfx950 BF16 matrix cores (operands prepared in ssn_direction)
    ChainArgs c{};
    c.m = tp.m; c.l = l; c.ldp = chain_ldp(l); c.r0 = tp.r0; c.v = v;
    c.Bh = ctx->Bh; c.BhT = ctx->BhT; c.Bl = ctx->Bl; c.BlT = ctx->BlT; c.Hh = ctx->Hh; c.Hl = ctx->Hl;
    c.a = tp.a; c.mu = tp.mu; c.w = tp.w; c.complement = tp.comp ? 1 : 0; c.diag_scale = 1.0; c.off_scale = 2.0;
    c.D = ctx->Bf + (long long)tp.r0 * l; c.ldd = l; c.alpha = tp.comp ? -1.0 : 1.0; c.part = ctx->part; c.y = y;
    HIPCHK(chain_bf16(c, mode == 2, st));
    return KOT_OK;
  }
  const float* Bs = ctx->Bf + (long long)tp.r0 * l;
  LowpArgs g{};
  g.m = tp.m; g.n = l; g.k = l; g.A = Bs; g.lda = l; g.s = v; g.B = ctx->Bf; g.ldb = l; g.transb = 1;
  g.C = ctx->Cf; g.ldc = l; g.l = l; g.a = tp.a; g.r0 = tp.r0; g.mu = tp.mu; g.w = tp.w; g.complement = tp.comp ? 1 : 0;
  g.diag_scale = 1.0; g.off_scale = 2.0;
  HIPCHK(gemm_lowp(g, mode, true, st));                 // H = Psi o (B_set diag(v) B^T)
  LowpArgs g2{};
  g2.m = tp.m; g2.n = l; g2.k = l; g2.A = ctx->Cf; g2.lda = l; g2.s = nullptr; g2.B = ctx->Bf; g2.ldb = l; g2.transb = 0;
  g2.C = ctx->Ef; g2.ldc = l;
  HIPCHK(gemm_lowp(g2, mode, false, st));               // E = H B
  HIPCHK(diag_dot_lowp(tp.m, l, tp.comp ? -1.0 : 1.0, Bs, l, ctx->Ef, l, y, ctx->part, st));
  return KOT_OK;
}

struct DirInfo {
  int cg_iters = 0;
  double cg_res = 0.0;
  int sweeps = 0;
  bool lowp = false;  // the reduced-precision chain ran
};

// Algorithm 1 at state s with regularization mu: writes ctx->dg, ctx->dX.
kot_status ssn_direction(kot_ctx* ctx, const CoreView& cv, const State& s, double mu, const kot_params* p, DirInfo* info) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  TPlan tp = make_tplan(l, s.a, mu, s.P, s.s);
  // B = P^T R
  if (cv.rd) HIPCHK(transpose_scale(l, s.P, cv.rd, ctx->Bm, st));
  else HIPCHK(mm(st, 1, 0, l, l, l, 1.0, s.P, l, nullptr, cv.R, l, 0.0, ctx->Bm, l, TRI_B_UPPER));
  // M = r2 + T[r2]  (kept in Mr), a1 = -r1 - Phi(M)/(mu+1)
  KCHK(t_apply(ctx, tp, s.r2, ctx->T1));
  HIPCHK(vec_lincomb(l * l, 1.0, s.r2, 1.0, ctx->T1, ctx->Mr, st));
  HIPCHK(vec_copy(l, s.r1, ctx->a1, st));
  KCHK(phi_op(ctx, cv, ctx->Mr, -1.0 / (mu + 1.0), -1.0, ctx->a1));
  const double* dinv = nullptr;
  if (p->precond == KOT_PRECOND_JACOBI) {
    KCHK(schur_dinv(ctx, cv, tp, ctx->cdinv));
    dinv = ctx->cdinv;
  }
  // CG on the Schur system from x = 0 (Eq. 4.5 on the CG residual), preconditioned when dinv is set
  double* x = ctx->cx;
  double* r = ctx->cr;
  double* pp = ctx->cp;
  double* Ap = ctx->cAp;
  const double rnorm = s.rn;
  int it = 0;
  double rr = 0.0;
  info->lowp = p->precision != KOT_FP64 && tp.m >= p->lowp_min_rows;
  double* cs = ctx->dsc + SL_CG;        // device CG state
  const double* hcs = ctx->hsc + SL_CG;
  const double kr = p->kappa * rnorm;
  const int cap = std::max(0, p->cg_max_iter);
  // CG on the device: iterations go out in batches between host checks of the stop flag (those queued past
  // the stop change nothing); one synchronization per batch instead of one per iteration
  // With schur_solver SQMR the same loop runs symmetric QMR (po is its direction q, Apo its product).
  const bool sqmr = p->schur_solver == KOT_SCHUR_SQMR;
  auto run_cg = [&](auto&& matvec, const double* b, double* xo, double* ro, double* po, double* Apo, double fixed,
                    int capc) -> kot_status {
    if (sqmr) HIPCHK(sqmr_init(l, b, xo, ro, po, ctx->qd, ctx->qe, ctx->qs, cs, p->tau, kr, fixed, capc, st, dinv));
    else HIPCHK(cg_init(l, b, xo, ro, po, cs, p->tau, kr, fixed, capc, st, dinv));
    for (int batch = 2;; batch = 3) {
      for (int q = 0; q < batch; ++q) {
        KCHK(matvec(po, Apo));
        if (sqmr)
          HIPCHK(sqmr_tail(l, cs, po, Apo, xo, ro, ctx->qd, ctx->qe, ctx->qs, p->tau, kr, fixed, capc, st, dinv));
        else
          HIPCHK(cg_tail(l, cs, po, Apo, 0.0, xo, ro, p->tau, kr, fixed, capc, st, dinv));
      }
      KCHK(sync_read(ctx));
      if (hcs[kCgDone] != 0.0) return KOT_OK;
    }
  };
  if (!info->lowp) {
    KCHK(run_cg([&](const double* v, double* y) { return schur_matvec(ctx, cv, tp, v, y); }, ctx->a1, x, r, pp, Ap,
                0.0, cap));
    it = (int)hcs[kCgIt];
    rr = hcs[kCgRR];
  } else {
    // Iterative refinement: each sweep solves M~ d = r with CG whose chain runs in reduced precision, then
    // x += d and the true residual r = a1 - M x is recomputed in FP64; Eq. 4.5 is checked on that residual.
    const int mode = p->precision == KOT_MIXED_BF16 ? 1 : (p->precision == KOT_MIXED_BF16X3 ? 2 : 0);
    const double inner_rel = mode == 1 ? 1e-2 : 1e-4;
    HIPCHK(f64_to_f32((long long)l * l, ctx->Bm, ctx->Bf, st));
    if (mode != 0)
      HIPCHK(chain_prep(l, chain_ldp(l), ctx->Bm, ctx->Bh, ctx->BhT, mode == 2 ? ctx->Bl : nullptr,
                        mode == 2 ? ctx->BlT : nullptr, st));
    HIPCHK(vec_fill(l, 0.0, x, st));
    HIPCHK(vec_copy(l, ctx->a1, r, st));
    double xx = 0.0;
    int sweeps = 0;
    while (true) {
      HIPCHK(dot2(l, r, r, ctx->dsc + SL_RR, x, x, ctx->dsc + SL_XX, ctx->part, st));
      KCHK(sync_read(ctx));
      rr = ctx->hsc[SL_RR];
      xx = ctx->hsc[SL_XX];
      const double thr = p->tau * std::min(1.0, kr * std::sqrt(xx));
      // the inner iterations of all sweeps share the CG cap of Remark 4.5 (cg_max_iter per direction)
      const int budget = std::max(1, p->cg_max_iter);
      if (std::sqrt(rr) <= thr || sweeps >= 8 || it >= budget) break;
      // inner CG from d = 0 on the reduced-precision operator, to a fixed threshold
      const double stop_in = std::max(inner_rel * std::sqrt(rr), 0.5 * thr);
      KCHK(run_cg([&](const double* v, double* y) { return schur_matvec_lowp(ctx, cv, tp, v, y, mode); }, r,
                  ctx->lx, ctx->lr, ctx->lp, ctx->lAp, stop_in, budget - it));
      it += (int)hcs[kCgIt];
      HIPCHK(vec_axpby(l, 1.0, ctx->lx, 1.0, x, st));
      KCHK(schur_matvec(ctx, cv, tp, x, Ap));                 // FP64 residual
      HIPCHK(vec_lincomb(l, 1.0, ctx->a1, -1.0, Ap, r, st));
      ++sweeps;
    }
    info->sweeps = sweeps;
  }
  info->cg_iters = it;
  info->cg_res = std::sqrt(rr);
  // dgamma = x;  dX = a~2 - T[Phi*(x)],  a~2 = (a2 + T[a2])/(mu+1) = -M/(mu+1)
  HIPCHK(vec_copy(l, x, ctx->dg, st));
  KCHK(phi_star(ctx, cv, x, ctx->T1));
  KCHK(t_apply(ctx, tp, ctx->T1, ctx->T2));
  HIPCHK(vec_lincomb(l * l, -1.0 / (mu + 1.0), ctx->Mr, -1.0, ctx->T2, ctx->dX, st));
  return KOT_OK;
}

// Pi(Y) into out via an eigendecomposition warm-started from Pbasis (updated in place); Y symmetric; wbuf: w.
kot_status proj_psd(kot_ctx* ctx, int l, double* Y, double* Pbasis, double* wbuf, bool warm, double* out,
                    const kot_params* p, int* sweeps_acc) {
  int a = 0;
  KCHK(eig_run(ctx, l, Y, warm ? Pbasis : nullptr, Pbasis, wbuf, p, sweeps_acc, &a));  // P0 may alias P
  KCHK(proj_from_eig(ctx, l, Y, Pbasis, wbuf, a, out));
  return KOT_OK;
}

// Pi(X - eta (Phi*(gs) + lam1 I)) into out, through the eigendecomposition (warm basis Pbasis, eigenvalues sbuf).
kot_status eg_proj(kot_ctx* ctx, const CoreView& cv, const double* gs, const double* X, double eta, double* Pbasis,
                   double* sbuf, bool warm, double* out, const kot_params* p, int* sweeps_acc) {
  const int l = cv.l;
  KCHK(phi_star(ctx, cv, gs, ctx->T1));
  HIPCHK(form_z(l, X, eta, ctx->T1, -eta * cv.lam1, ctx->Z, ctx->stream));
  KCHK(proj_psd(ctx, l, ctx->Z, Pbasis, sbuf, warm, out, p, sweeps_acc));
  return KOT_OK;
}

// One extragradient step on Eq. (4.1) from (g, X) with r1(g, X) given; writes (gn, Xn):
//   gh = g - eta r1(g, X),  Xh = Pi(X - eta (Phi*(g) + lam1 I)),  gn = g - eta r1(gh, Xh),
//   Xn = Pi(X - eta (Phi*(gh) + lam1 I)).
// The X-part of the operator depends on gamma alone, so Xn needs gh but not Xh: the two projections are
// independent (the overlapped iteration runs them on two streams).  When warm, both start from the previous
// step's bases, the first from the second's: X is then Pi of the matrix that basis diagonalizes, and the matrix
// projected first differs from that one by its negative part (diagonal in the basis) and an eta-sized term.
kot_status eg_step_impl(kot_ctx* ctx, const CoreView& cv, const double* g, const double* X, const double* r1,
                        double eta, double* gn, double* Xn, bool warm, const kot_params* p, int* sweeps_acc) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  HIPCHK(vec_lincomb(l, 1.0, g, -eta, r1, ctx->gh, st));
  if (warm) HIPCHK(vec_copy(l * l, ctx->Pe2, ctx->Pe1, st));
  KCHK(eg_proj(ctx, cv, g, X, eta, ctx->Pe1, ctx->s_e1, warm, ctx->Xh, p, sweeps_acc));
  KCHK(r1_op(ctx, cv, ctx->gh, ctx->Xh, ctx->r1h));
  HIPCHK(vec_lincomb(l, 1.0, g, -eta, ctx->r1h, gn, st));
  KCHK(eg_proj(ctx, cv, ctx->gh, X, eta, ctx->Pe2, ctx->s_e2, warm, Xn, p, sweeps_acc));
  return KOT_OK;
}

kot_status copy_state(kot_ctx* ctx, int l, const State& from, State& to) {
  hipStream_t st = ctx->stream;
  HIPCHK(vec_copy(l, from.g, to.g, st));
  HIPCHK(vec_copy(l * l, from.X, to.X, st));
  HIPCHK(vec_copy(l, from.r1, to.r1, st));
  HIPCHK(vec_copy(l * l, from.r2, to.r2, st));
  HIPCHK(vec_copy(l * l, from.P, to.P, st));
  HIPCHK(vec_copy(l, from.s, to.s, st));
  to.a = from.a; to.r1n = from.r1n; to.r2n = from.r2n; to.rn = from.rn; to.has_eig = from.has_eig;
  return KOT_OK;
}

kot_status prepare_core(kot_ctx* ctx, CoreView& cv) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  // KK = (R^T R) o (R^T R); after the setup R^T R = K + eps I is at hand without the product
  if (cv.kb_state == 0)
    HIPCHK(mm(st, 1, 0, l, l, l, 1.0, cv.R, l, nullptr, cv.R, l, 0.0, ctx->Kb, l, TRI_A_LOWER | TRI_B_UPPER, true));
  if (cv.kb_state < 2) HIPCHK(hadamard_square(l * l, ctx->Kb, ctx->KKb, st));
  cv.kb_state = 2;
  cv.KK = ctx->KKb;
  return KOT_OK;
}

// Default EG step (Section 4.2): eta = 1 / (2 L) with L bounded by |Q|_inf/(2 lam2) + sqrt(|K o K|_inf).  The
// row-sum maxima go to the SL_ETA slots; default_eta_read takes them after a later sync_read.
kot_status default_eta_launch(kot_ctx* ctx, const CoreView& cv) {
  const int l = cv.l;
  HIPCHK(rowsum_abs_max(l, cv.Q, false, ctx->dsc + SL_ETA, ctx->part, ctx->stream));
  HIPCHK(rowsum_abs_max(l, cv.KK, false, ctx->dsc + SL_ETA + 1, ctx->part, ctx->stream));
  return KOT_OK;
}
double default_eta_value(double qmax, double kkmax, double lam2) {
  return 0.5 / (qmax / (2.0 * lam2) + std::sqrt(kkmax));
}
double default_eta_read(kot_ctx* ctx, const CoreView& cv) {
  return default_eta_value(ctx->hsc[SL_ETA], ctx->hsc[SL_ETA + 1], cv.lam2);
}

kot_status check_params(kot_ctx* ctx, const kot_params* p, bool need_sigma) {
  if (!p) return fail(ctx, KOT_ERR_ARG, "params is NULL");
  if (need_sigma && !(p->sigma > 0.0)) return fail(ctx, KOT_ERR_ARG, "sigma must be > 0");
  if (!(p->lambda1 > 0.0) || !(p->lambda2 > 0.0)) return fail(ctx, KOT_ERR_ARG, "lambda1, lambda2 must be > 0");
  if (p->max_iter < 0 || p->cg_max_iter < 0) return fail(ctx, KOT_ERR_ARG, "negative iteration cap");
  if (p->precision != KOT_FP64 && p->precision != KOT_FP32 && p->precision != KOT_MIXED_BF16 &&
      p->precision != KOT_MIXED_BF16X3)
    return fail(ctx, KOT_ERR_ARG, "unknown precision %d", p->precision);
  if (p->safeguard != KOT_SAFEGUARD_EG && p->safeguard != KOT_SAFEGUARD_NONE && p->safeguard != KOT_SAFEGUARD_EG_ONLY)
    return fail(ctx, KOT_ERR_ARG, "unknown safeguard %d", p->safeguard);
  if (p->lowp_min_rows < 0) return fail(ctx, KOT_ERR_ARG, "lowp_min_rows must be >= 0");
  if (p->precond != KOT_PRECOND_NONE && p->precond != KOT_PRECOND_JACOBI)
    return fail(ctx, KOT_ERR_ARG, "precond must be KOT_PRECOND_NONE or KOT_PRECOND_JACOBI");
  if (p->schur_solver != KOT_SCHUR_CG && p->schur_solver != KOT_SCHUR_SQMR)
    return fail(ctx, KOT_ERR_ARG, "schur_solver must be KOT_SCHUR_CG or KOT_SCHUR_SQMR");
  if (p->closed_start < 0 || p->closed_start > 2) return fail(ctx, KOT_ERR_ARG, "closed_start must be 0, 1 or 2");
  return KOT_OK;
}

kot_status ensure_mlp(kot_ctx* ctx, size_t rows, size_t H, size_t l) {
  const size_t need_rows = std::max(rows, l);
  if (need_rows <= ctx->mlp_rows && H <= ctx->mlp_h && ctx->rs3) return KOT_OK;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (void* p : ctx->mbufs) hipFree(p);
  ctx->mbufs.clear();
  const size_t R = std::max(need_rows, ctx->mlp_rows), Hh = std::max(H, ctx->mlp_h);
  auto falloc = [&](size_t n) -> float* {
    void* p = nullptr;
    if (hipMalloc(&p, n * sizeof(float)) != hipSuccess) return nullptr;
    ctx->mbufs.push_back(p);
    return (float*)p;
  };
  if (!(ctx->fA1 = falloc(R * Hh)) || !(ctx->fA2 = falloc(R * Hh)) || !(ctx->fdZ1 = falloc(R * Hh)) ||
      !(ctx->fdZ2 = falloc(R * Hh)) || !(ctx->fout = falloc(R)) || !(ctx->fdout = falloc(R)) ||
      !(ctx->fpart = falloc(16 * Hh + 16)) || !(ctx->fX = falloc(R * kFeatures)))
    return fail(ctx, KOT_ERR_OOM, "network workspace allocation failed");
  void* p = nullptr;
  if (hipMalloc(&p, 3 * R * sizeof(double)) != hipSuccess) return fail(ctx, KOT_ERR_OOM, "allocation failed");
  ctx->mbufs.push_back(p);
  ctx->rs3 = (double*)p;
  ctx->mlp_rows = R;
  ctx->mlp_h = Hh;
  return KOT_OK;
}

struct MlpView {
  int F, H;
  const float *W1, *b1, *W2, *b2, *W3, *b3;
};
MlpView mlp_view(int F, int H, const float* th) {
  MlpView v;
  v.F = F; v.H = H;
  v.W1 = th; v.b1 = v.W1 + (size_t)F * H; v.W2 = v.b1 + H; v.b2 = v.W2 + (size_t)H * H; v.W3 = v.b2 + H; v.b3 = v.W3 + H;
  return v;
}
GemmF32Args g32(int ta, int tb, int m, int n, int k, const float* A, int lda, const float* B, int ldb, float* C, int ldc,
                const float* bias = nullptr, int act = 0, const float* mask = nullptr, int ldm = 0) {
  GemmF32Args g{};
  g.ta = ta; g.tb = tb; g.m = m; g.n = n; g.k = k; g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.beta = 0.f; g.bias = bias; g.act = act; g.mask = mask; g.ldm = ldm;
  return g;
}

kot_status mlp_forward_impl(kot_ctx* ctx, int n, const MlpView& w, const float* X, float* out) {
  hipStream_t st = ctx->stream;
  const int F = w.F, H = w.H;
  HIPCHK(gemm_f32(g32(0, 0, n, H, F, X, F, w.W1, H, ctx->fA1, H, w.b1, 1), st));
  HIPCHK(gemm_f32(g32(0, 0, n, H, H, ctx->fA1, H, w.W2, H, ctx->fA2, H, w.b2, 1), st));
  HIPCHK(gemm_f32(g32(0, 0, n, 1, H, ctx->fA2, H, w.W3, 1, out, 1, w.b3, 0), st));
  return KOT_OK;
}

kot_status mlp_loss_grad_impl(kot_ctx* ctx, int n, const MlpView& w, const float* X, const float* y, float* grad,
                              double* loss) {
  hipStream_t st = ctx->stream;
  const int F = w.F, H = w.H;
  KCHK(mlp_forward_impl(ctx, n, w, X, ctx->fout));
  HIPCHK(mse_grad(n, ctx->fout, y, ctx->fdout, ctx->dsc + 0, ctx->part, st));
  float* gW1 = grad;
  float* gb1 = gW1 + (size_t)F * H;
  float* gW2 = gb1 + H;
  float* gb2 = gW2 + (size_t)H * H;
  float* gW3 = gb2 + H;
  float* gb3 = gW3 + H;
  HIPCHK(gemm_f32(g32(1, 0, H, 1, n, ctx->fA2, H, ctx->fdout, 1, gW3, 1), st));
  HIPCHK(colsum_f32(n, 1, ctx->fdout, gb3, ctx->fpart, st));
  HIPCHK(gemm_f32(g32(0, 1, n, H, 1, ctx->fdout, 1, w.W3, 1, ctx->fdZ2, H, nullptr, 0, ctx->fA2, H), st));
  HIPCHK(gemm_f32(g32(1, 0, H, H, n, ctx->fA1, H, ctx->fdZ2, H, gW2, H), st));
  HIPCHK(colsum_f32(n, H, ctx->fdZ2, gb2, ctx->fpart, st));
  HIPCHK(gemm_f32(g32(0, 1, n, H, H, ctx->fdZ2, H, w.W2, H, ctx->fdZ1, H, nullptr, 0, ctx->fA1, H), st));
  HIPCHK(gemm_f32(g32(1, 0, F, H, n, X, F, ctx->fdZ1, H, gW1, H), st));
  HIPCHK(colsum_f32(n, H, ctx->fdZ1, gb1, ctx->fpart, st));
  KCHK(sync_read(ctx, 1, 0));
  *loss = ctx->hsc[0];
  return KOT_OK;
}

// gamma0 = lambda1 * f(features) for the prepared core (KK must be set).
// K: the buffer holding R^T R (K + eps I)
kot_status predict_gamma0(kot_ctx* ctx, const CoreView& cv, const double* K, int F, int H, const float* theta,
                          double* gamma0) {
  const int l = cv.l;
  if (F != kFeatures) return fail(ctx, KOT_ERR_ARG, "the feature map has %d features (got F=%d)", kFeatures, F);
  KCHK(ensure_mlp(ctx, l, H, l));
  HIPCHK(features(l, cv.Q, cv.z, cv.wsum, K, cv.KK, cv.lam1, ctx->rs3, ctx->dsc + SL_POOL, ctx->fX, ctx->stream));
  KCHK(mlp_forward_impl(ctx, l, mlp_view(F, H, theta), ctx->fX, ctx->fout));
  HIPCHK(f32_to_f64_scaled(l, ctx->fout, cv.lam1, gamma0, ctx->stream));
  return KOT_OK;
}

// ---- the extragradient branch on a second stream ---------------------------------------------------------
// In each iteration of Algorithm 2 the extragradient iterate v_{k+1} and its residual depend only on v_k, and
// the Newton trial only on w_k: the branches meet in the accept test alone, so they can run concurrently.  A
// child context (own stream, workspace and eigensolver state) runs the extragradient branch from a host
// thread of its own while the calling thread runs the Newton branch; the kernels and their inputs are the
// same as on one stream, so are the iterates.  Between jobs the thread spins for a few milliseconds (the next
// job of a solve comes within that), then sleeps on a condition variable.
struct SideRunner {
  kot_ctx* c = nullptr;
  std::thread th;
  std::mutex mu;
  std::condition_variable cvar;
  std::atomic<int> state{0};  // 0 idle, 1 job posted, 2 job done
  std::atomic<bool> quit{false};
  std::function<kot_status()> job;
  kot_status rc = KOT_OK;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at a post; the side stream waits for it
};

void bind_thread(kot_ctx* c) {
  g_prof = &c->prof;
  g_gemm_ws = c->gemm_ws;
  g_gemm_ws_cap = c->gemm_ws_cap;
  g_gemm_tune = c->tuned ? c->tune : nullptr;
}

void side_loop(SideRunner* s) {
  using clk = std::chrono::steady_clock;
  for (;;) {
    const auto t0 = clk::now();
    int spins = 0;
    while (s->state.load(std::memory_order_acquire) != 1) {
      if (s->quit.load(std::memory_order_acquire)) return;
      if (++spins >= 256) {
        spins = 0;
        if (clk::now() - t0 > std::chrono::milliseconds(5)) {
          std::unique_lock<std::mutex> lk(s->mu);
          s->cvar.wait(lk, [s] { return s->quit.load() || s->state.load() == 1; });
          continue;
        }
      }
      __builtin_ia32_pause();
    }
    kot_ctx* c = s->c;
    bind_thread(c);
    kot_status rc;
    hipError_t e = hipSetDevice(c->device);
    if (e == hipSuccess) {
      e = hipStreamWaitEvent(c->stream, s->ready, 0);
      if (e != hipSuccess) {  // a device-side wait that could not be queued: wait on the host (same ordering)
        (void)hipGetLastError();
        e = hipEventSynchronize(s->ready);
      }
    }
    if (e != hipSuccess)
      rc = fail(c, KOT_ERR_HIP, "could not order the side stream after the caller's stream (%s)", hipGetErrorString(e));
    else
      rc = s->job();
    s->rc = rc;
    s->state.store(2, std::memory_order_release);
  }
}

kot_status runner_ensure(kot_ctx* ctx, SideRunner** slot, int l, int nmax) {
  if (!*slot) {
    SideRunner* s = new SideRunner();
    kot_ctx* c = nullptr;
    const kot_status st = kot_create(&c, ctx->device, nullptr);
    if (st != KOT_OK) {
      delete s;
      return fail(ctx, st, "could not create a side context");
    }
    s->c = c;
    if (hipEventCreateWithFlags(&s->ready, hipEventDisableTiming) != hipSuccess) {
      kot_destroy(c);
      delete s;
      return fail(ctx, KOT_ERR_HIP, "could not create a side event");
    }
    s->th = std::thread(side_loop, s);
    *slot = s;
  }
  kot_ctx* c = (*slot)->c;
  c->tuned = ctx->tuned;
  if (ctx->tuned) std::copy(ctx->tune, ctx->tune + kTuneBuckets, c->tune);
  const kot_status st = ensure_ws(c, l, nmax);
  bind_thread(ctx);  // ensure_ws binds the calling thread to the context it sizes
  if (st < 0) return fail(ctx, st, "side workspace: %s", c->err.c_str());
  return KOT_OK;
}

kot_status side_ensure(kot_ctx* ctx, int l, int nmax) {
  KCHK(runner_ensure(ctx, &ctx->side, l, nmax));
  return runner_ensure(ctx, &ctx->side2, l, 0);
}

// Queues f on runner s, ordered after the work queued so far on ctx's stream.
kot_status runner_post(kot_ctx* ctx, SideRunner* s, std::function<kot_status()> f) {
  HIPCHK(hipEventRecord(s->ready, ctx->stream));
  s->c->prof.on = ctx->prof.on;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->job = std::move(f);
    s->state.store(1, std::memory_order_release);
  }
  s->cvar.notify_one();
  return KOT_OK;
}
kot_status side_post(kot_ctx* ctx, std::function<kot_status()> f) { return runner_post(ctx, ctx->side, std::move(f)); }

// Waits for the job posted on s (from whichever thread posted it); on return the side stream has finished all
// of the job's work (every job ends with a host synchronization of its stream).  Errors are reported on ctx.
kot_status runner_join(kot_ctx* ctx, SideRunner* s) {
  while (s->state.load(std::memory_order_acquire) != 2) __builtin_ia32_pause();
  s->state.store(0, std::memory_order_relaxed);
  s->job = nullptr;
  if (s->rc < 0) return fail(ctx, s->rc, "second stream: %s", s->c->err.c_str());
  return KOT_OK;
}
kot_status side_join(kot_ctx* ctx) { return runner_join(ctx, ctx->side); }

void runner_destroy(SideRunner*& s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->quit.store(true, std::memory_order_release);
  }
  s->cvar.notify_one();
  if (s->th.joinable()) s->th.join();
  if (s->ready) hipEventDestroy(s->ready);
  kot_destroy(s->c);
  delete s;
  s = nullptr;
}
void side_destroy(kot_ctx* ctx) {
  runner_destroy(ctx->side);
  runner_destroy(ctx->side2);
}

constexpr int kOverlapMinL = 128;

bool overlap_ok(const kot_ctx* ctx, const kot_params* p, int l) {
  return p->overlap && l >= kOverlapMinL && !ctx->is_lane;
}

// Algorithm 2 on a prepared core.
// Y = R^-1 (W: workspace) through a HIP graph of the launches of trtri_upper, captured on the first call for
// these buffers (that call runs them directly, which also builds any GEMM work list they need) and replayed
// afterwards.  With the profiler on, or when capture fails, the launches go out one by one.
kot_status trtri_cached(kot_ctx* ctx, int l, const double* R, double* Y, double* W) {
  hipStream_t st = ctx->stream;
  const void* key[4] = {R, Y, W, g_gemm_ws};
  const bool same = ctx->trtri_graph && ctx->trtri_l == l && std::equal(key, key + 4, ctx->trtri_key);
  if (same && !(g_prof && g_prof->on)) {
    HIPCHK(hipGraphLaunch(ctx->trtri_graph, st));
    return KOT_OK;
  }
  HIPCHK(trtri_upper(l, R, Y, W, st));
  if (ctx->trtri_graph_failed || (g_prof && g_prof->on)) return KOT_OK;
  if (ctx->trtri_graph) {
    hipGraphExecDestroy(ctx->trtri_graph);
    ctx->trtri_graph = nullptr;
  }
  hipGraph_t gr = nullptr;
  bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    const hipError_t le = trtri_upper(l, R, Y, W, st);
    ok = hipStreamEndCapture(st, &gr) == hipSuccess && le == hipSuccess && gr != nullptr;
  }
  if (ok) ok = hipGraphInstantiate(&ctx->trtri_graph, gr, nullptr, nullptr, 0) == hipSuccess;
  if (gr) hipGraphDestroy(gr);
  if (!ok) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;  // a failed capture must not stay open
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) {
      hipGraph_t g2 = nullptr;
      (void)hipStreamEndCapture(st, &g2);
      if (g2) hipGraphDestroy(g2);
    }
    (void)hipGetLastError();
    ctx->trtri_graph = nullptr;
    ctx->trtri_graph_failed = true;
    return KOT_OK;
  }
  ctx->trtri_l = l;
  std::copy(key, key + 4, ctx->trtri_key);
  return KOT_OK;
}

// pre: the setup already formed KK, the default step's bounds, |z|^2 and the network's start (in S[1].g).
kot_status run_alg2(kot_ctx* ctx, CoreView& cv, const kot_params* p, const double* gamma0, kot_result* res,
                    const Prelude* pre = nullptr) {
  const int l = cv.l;
  hipStream_t st = ctx->stream;
  HIPCHK(hipEventRecord(ctx->ev0, st));
  KCHK(prepare_core(ctx, cv));
  double eta = p->eg_step;
  const bool eta_default = !(eta > 0.0);
  if (!pre) {
    if (eta_default) KCHK(default_eta_launch(ctx, cv));       // read with the first residual's norms
    if (gamma0 || p->ws_theta || p->closed_start == 1) HIPCHK(dot(l, cv.z, cv.z, ctx->dsc + SL_ZZ, ctx->part, st));
  }
  State* W = &ctx->S[0];
  State* T = &ctx->S[1];
  State* V = &ctx->S[2];
  if (p->ws_theta && !gamma0) {  // learned start
    if (!pre) KCHK(predict_gamma0(ctx, cv, ctx->Kb, p->ws_F, p->ws_H, p->ws_theta, ctx->S[1].g));
    gamma0 = ctx->S[1].g;
  } else if (p->closed_start == 1 && !gamma0) {  // closed-form start (the diagonal, orthogonal-factor minimizer)
    HIPCHK(closed_start(l, cv.Q, cv.z, cv.lam1, ctx->S[1].g, st));
    gamma0 = ctx->S[1].g;
  }
  if (gamma0) HIPCHK(vec_copy(l, gamma0, W->g, st));
  else HIPCHK(vec_fill(l, 0.0, W->g, st));
  // X0 for the start in W->g: with lift_x0, X0 = R^-T diag(y) R^-1 with y = (Q gamma0 - z)/(2 lam2)
  // (stationarity's value of Phi(X)) on the constraints predicted active, small entries dropped, so that
  // Phi(X0) = y; else X0 = 0
  auto start_x = [&]() -> kot_status {
    if (!p->lift_x0) {
      HIPCHK(vec_fill(l * l, 0.0, W->X, st));
      return KOT_OK;
    }
    if (!cv.Linv && !cv.rd) KCHK(trtri_cached(ctx, l, cv.R, ctx->T1, ctx->T2));
    HIPCHK(mm(st, 0, 0, l, 1, l, 1.0, cv.Q, l, nullptr, W->g, 1, 0.0, ctx->vtmp, 1));
    HIPCHK(lift_diag(l, ctx->vtmp, cv.z, W->g, cv.lam1, cv.lam2, 0.02, ctx->dg, ctx->part, st));
    if (cv.rd)
      HIPCHK(diag_gram(l, cv.rd, -2, ctx->dg, W->X, st));
    else if (cv.Linv)
      HIPCHK(mm(st, 0, 1, l, l, l, 1.0, cv.Linv, l, ctx->dg, cv.Linv, l, 0.0, W->X, l, TRI_A_LOWER | TRI_B_UPPER,
                true));
    else
      HIPCHK(mm(st, 1, 0, l, l, l, 1.0, ctx->T1, l, ctx->dg, ctx->T1, l, 0.0, W->X, l, TRI_A_LOWER | TRI_B_UPPER,
                true));
    return KOT_OK;
  };
  if (gamma0) KCHK(start_x());
  else HIPCHK(vec_fill(l * l, 0.0, W->X, st));
  int sweeps = 0;
  // Fallback test of a start w0: kept when |R(w0)| <= |R(0, 0)| = |z|/(2 lam2) (Pi(-lambda1 I) = 0), else the
  // cold start is taken.  |R(w0)| >= |r1(w0)|, and r1 needs no eigendecomposition: a start whose r1 alone exceeds
  // the bound (by more than the two norms' rounding) is dropped before its Z is decomposed, with the same outcome.
  auto test_start = [&](bool* kept) -> kot_status {
    KCHK(r1_op(ctx, cv, W->g, W->X, W->r1));
    HIPCHK(dot(l, W->r1, W->r1, ctx->dsc + SL_R1, ctx->part, st));
    KCHK(sync_read(ctx));
    const double cold = std::sqrt(pre ? pre->zz : ctx->hsc[SL_ZZ]) / (2.0 * cv.lam2);
    *kept = false;
    if (!(std::sqrt(ctx->hsc[SL_R1]) <= cold * (1.0 + 1e-12))) return KOT_OK;
    KCHK(residual_state(ctx, cv, *W, nullptr, p, &sweeps));
    *kept = W->rn <= cold;
    return KOT_OK;
  };
  res->warm_used = 0;
  bool kept = false;
  if (gamma0) {
    // With closed_start = 2 a rejected start (the network's or the caller's) is first replaced by the
    // closed-form start, which is kept on the same test.
    KCHK(test_start(&kept));
    if (kept) {
      res->warm_used = 1;
    } else if (p->closed_start == 2) {
      HIPCHK(closed_start(l, cv.Q, cv.z, cv.lam1, W->g, st));
      KCHK(start_x());
      KCHK(test_start(&kept));
      if (kept) res->warm_used = 2;
    }
    if (!kept) {
      HIPCHK(vec_fill(l, 0.0, W->g, st));
      HIPCHK(vec_fill(l * l, 0.0, W->X, st));
    }
  }
  if (!kept) KCHK(residual_state(ctx, cv, *W, nullptr, p, &sweeps));
  if (eta_default) eta = pre ? pre->eta : default_eta_read(ctx, cv);
  const bool use_eg = p->safeguard == KOT_SAFEGUARD_EG;
  const bool overlap = use_eg && overlap_ok(ctx, p, l);
  int side_sweeps = 0, side2_sweeps = 0;
  if (overlap) KCHK(side_ensure(ctx, l, 0));
  // v_0 = w_0 without a copy: the first extragradient step reads w_0's buffers (which nothing writes before the
  // accept test) and writes v_1 into V's own; only the host-side norms are copied
  if (use_eg) {
    V->a = W->a; V->r1n = W->r1n; V->r2n = W->r2n; V->rn = W->rn; V->has_eig = W->has_eig;
  }
  double theta = p->theta0;
  bool v_basis = false;  // V->P holds an eigenbasis (written by a full residual at a v)
  int k = 0, cg_total = 0, eg_acc = 0, nulls = 0, lowp_dirs = 0;
  kot_status status = KOT_NOT_CONVERGED;
  bool warm_e = false;
  for (k = 0;; ++k) {
    if (res->res_hist && k < res->hist_cap) res->res_hist[k] = W->rn;
    if (res->res_v_hist && k < res->hist_cap) res->res_v_hist[k] = use_eg ? V->rn : W->rn;
    if (!std::isfinite(W->rn)) { status = KOT_ERR_NUMERIC; break; }
    if (W->rn <= p->tol) { status = KOT_OK; break; }
    if (k >= p->max_iter) break;
    if (p->safeguard == KOT_SAFEGUARD_EG_ONLY) {  // pure extragradient: w_{k+1} = EG step from w_k
      State* H = &ctx->S[3];
      KCHK(eg_step_impl(ctx, cv, W->g, W->X, W->r1, eta, H->g, H->X, warm_e && p->warm_eig, p, &sweeps));
      warm_e = true;
      std::swap(H->g, W->g);
      std::swap(H->X, W->X);
      KCHK(residual_state(ctx, cv, *W, p->warm_eig ? W->P : nullptr, p, &sweeps));
      continue;
    }
    // (1) safeguard: one EG step from v_k (w_0 at k = 0), then r1 at v_{k+1} (its full residual only if the
    // accept test needs it, below); on the side streams when overlapped
    const State* Vs = k == 0 ? W : V;
    // warm basis of the residual at v_{k+1} (when it is needed): V's own last eigenbasis once one has been
    // computed, else w_k's (V's buffer holds no basis before the first full residual at a v)
    const double* Pv = !p->warm_eig ? nullptr : (k > 0 && v_basis ? V->P : W->P);
    if (use_eg && overlap) {
      // gh on this stream, then the projection for Xn on the third stream and the rest of the branch (the
      // projection for Xh, gn, r1 at v_{k+1} once Xn is in) on the second
      const bool warm_v = warm_e && p->warm_eig;
      State* H = &ctx->S[3];
      HIPCHK(vec_lincomb(l, 1.0, Vs->g, -eta, Vs->r1, ctx->gh, st));
      // the first projection starts from the second's basis of the previous step, as in the one-stream order;
      // copied on this stream, so before the third stream's job (ordered after it) overwrites that basis
      if (warm_v) HIPCHK(vec_copy(l * l, ctx->side2->c->Pe2, ctx->side->c->Pe1, st));
      KCHK(runner_post(ctx, ctx->side2, [ctx, &cv, Vs, H, eta, warm_v, p, &side2_sweeps]() -> kot_status {
        kot_ctx* c = ctx->side2->c;
        KCHK(eg_proj(c, cv, ctx->gh, Vs->X, eta, c->Pe2, c->s_e2, warm_v, H->X, p, &side2_sweeps));
        if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(c, KOT_ERR_HIP, "stream synchronization");
        return KOT_OK;
      }));
      const kot_status rp = side_post(ctx, [ctx, &cv, Vs, V, H, eta, warm_v, p, &side_sweeps]() -> kot_status {
        kot_ctx* c = ctx->side->c;
        const int n = cv.l;
        const kot_status r0 = eg_proj(c, cv, Vs->g, Vs->X, eta, c->Pe1, c->s_e1, warm_v, c->Xh, p, &side_sweeps);
        kot_status r1 = r0 < 0 ? r0 : r1_op(c, cv, ctx->gh, c->Xh, c->r1h);
        if (r1 >= 0 && vec_lincomb(n, 1.0, Vs->g, -eta, c->r1h, H->g, c->stream) != hipSuccess)
          r1 = fail(c, KOT_ERR_HIP, "vec_lincomb");
        const kot_status r2 = runner_join(c, ctx->side2);  // Xn (joined even after a failure)
        KCHK(r1);
        KCHK(r2);
        std::swap(H->g, V->g);
        std::swap(H->X, V->X);
        return r1_only(c, cv, *V);
      });
      if (rp < 0) {  // the third stream's job is already out: wait for it before returning
        (void)runner_join(ctx, ctx->side2);
        return rp;
      }
      warm_e = true;
    } else if (use_eg) {
      State* H = &ctx->S[3];
      KCHK(eg_step_impl(ctx, cv, Vs->g, Vs->X, Vs->r1, eta, H->g, H->X, warm_e && p->warm_eig, p, &sweeps));
      warm_e = true;
      std::swap(H->g, V->g);
      std::swap(H->X, V->X);
      KCHK(r1_only(ctx, cv, *V, false));
    }
    // (2) regularized SSN trial
    const double mu = theta * W->rn;
    DirInfo di;
    auto newton = [&]() -> kot_status {
      KCHK(ssn_direction(ctx, cv, *W, mu, p, &di));
      cg_total += di.cg_iters;
      lowp_dirs += di.lowp ? 1 : 0;
      HIPCHK(vec_lincomb(l, 1.0, W->g, 1.0, ctx->dg, T->g, st));
      HIPCHK(vec_lincomb(l * l, 1.0, W->X, 1.0, ctx->dX, T->X, st));
      KCHK(residual_state(ctx, cv, *T, p->warm_eig ? W->P : nullptr, p, &sweeps, SL_TN, true));
      // theta rule (Section 4.3): rho = -<R(w + dw), dw>; one host synchronization brings these dots and the
      // deferred residual norms of the trial and of the EG point
      HIPCHK(dot2(l, T->r1, ctx->dg, ctx->dsc + SL_THETA, ctx->dg, ctx->dg, ctx->dsc + SL_THETA + 2, ctx->part, st));
      HIPCHK(dot2((long long)l * l, T->r2, ctx->dX, ctx->dsc + SL_THETA + 1, ctx->dX, ctx->dX,
                  ctx->dsc + SL_THETA + 3, ctx->part, st));
      KCHK(sync_read(ctx));
      return KOT_OK;
    };
    const kot_status rc_newton = newton();
    if (use_eg && overlap) {
      const kot_status rc_side = side_join(ctx);  // joined even when the Newton branch failed
      sweeps += side_sweeps + side2_sweeps;
      side_sweeps = side2_sweeps = 0;
      KCHK(rc_newton);
      KCHK(rc_side);
    }
    KCHK(rc_newton);
    finish_norms(ctx, *T, SL_TN);
    if (use_eg) {
      // |R(v_{k+1})| >= |r1(v_{k+1})|: when the trial's residual is below that bound (by more than the norms'
      // rounding), the accept test below takes the trial (and the null-step variant's W->rn <= |R(v_{k+1})|
      // holds whenever it is asked) whatever r2 is, so the eigendecomposition of Z at v_{k+1} is not needed:
      // |R(v_{k+1})| is then recorded as that lower bound.  Otherwise the full residual is computed.
      const double r1v = std::sqrt(overlap ? ctx->side->c->hsc[SL_VN] : ctx->hsc[SL_VN]);
      if (T->rn <= r1v * (1.0 - 1e-12)) {
        V->r1n = r1v;
        V->r2n = 0.0;
        V->rn = r1v;
        V->has_eig = false;
      } else {
        KCHK(residual_state(ctx, cv, *V, Pv, p, &sweeps, SL_VN, false));
        v_basis = true;
      }
    }
    const double rho = -(ctx->hsc[SL_THETA] + ctx->hsc[SL_THETA + 1]);
    const double dwn = std::sqrt(ctx->hsc[SL_THETA + 2]) + std::sqrt(ctx->hsc[SL_THETA + 3]);
    const double dw2 = dwn * dwn;
    if (rho >= p->alpha2 * dw2) theta = std::max(p->theta_min, p->beta0 * theta);
    else if (rho >= p->alpha1 * dw2) theta = p->beta1 * theta;
    else theta = std::min(p->theta_max, p->beta2 * theta);
    // (3) accept test
    const double rv = use_eg ? V->rn : INFINITY;
    if (p->null_step && T->rn > W->rn && (!use_eg || W->rn <= rv)) {
      ++nulls;
    } else if (!use_eg || T->rn <= rv) {
      std::swap(ctx->S[0], ctx->S[1]);
      W = &ctx->S[0];
      T = &ctx->S[1];
    } else {
      KCHK(copy_state(ctx, l, *V, *W));
      ++eg_acc;
    }
  }
  res->iters = k;
  res->cg_iters_total = cg_total;
  res->lowp_directions = lowp_dirs;
  res->eg_accepts = eg_acc;
  res->null_steps = nulls;
  res->eig_sweeps_total = sweeps;
  res->alpha_last = W->a;
  res->residual = W->rn;
  // outputs
  if (res->gamma) HIPCHK(vec_copy(l, W->g, res->gamma, st));
  if (res->X) HIPCHK(vec_copy(l * l, W->X, res->X, st));
  HIPCHK(dot(l, W->g, cv.wsum, ctx->dsc + SL_TMP, ctx->part, st));
  HIPCHK(hipEventRecord(ctx->ev1, st));
  KCHK(sync_read(ctx));
  res->ot = (cv.q2 - ctx->hsc[SL_TMP]) / (2.0 * cv.lam2);
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  res->time_ms = ms;
  if (status == KOT_ERR_NUMERIC) return fail(ctx, KOT_ERR_NUMERIC, "non-finite residual at iteration %d", k);
  return status;
}

// Whether K + eps I (in ctx->Kb) is diagonal to kdiag_tol relative to its largest diagonal entry (a host
// synchronization); if so R = diag(sqrt(K_ii + eps)) (rd: its diagonal; Linv: R^-T) replaces the factorization.
kot_status kdiag_factor(kot_ctx* ctx, int l, const kot_params* p, double* R, double* rd, double* Linv, bool* diag) {
  *diag = false;
  if (!(p->kdiag_tol > 0.0) || !rd) return KOT_OK;
  HIPCHK(offdiag_absmax(l, ctx->Kb, ctx->dsc + SL_KD, ctx->stream));
  KCHK(sync_read(ctx));
  if (!(ctx->hsc[SL_KD] <= p->kdiag_tol * ctx->hsc[SL_KD + 1])) return KOT_OK;
  HIPCHK(diag_factor(l, ctx->Kb, R, rd, Linv, ctx->dint, ctx->stream));
  *diag = true;
  return KOT_OK;
}

// Linv (optional): receives R^-T from the factorization.  rd (optional): with kdiag_tol, the diagonal of a
// diagonal R (*diag set when taken).
kot_status setup_impl(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, double* Q, double* z, double* R,
                      double* wsum, double* q2, double* Linv = nullptr, double* rd = nullptr, bool* diag = nullptr) {
  const int l = pb->l, d = pb->d;
  hipStream_t st = ctx->stream;
  HIPCHK(gram_build(l, d, pb->xf, pb->yf, p->sigma, Q, ctx->Kb, st));
  HIPCHK(add_diag(l, p->eps_jitter, ctx->Kb, st));  // K + eps I = R^T R from here on
  bool dg = false;
  KCHK(kdiag_factor(ctx, l, p, R, rd, Linv, &dg));
  if (diag) *diag = dg;
  HIPCHK(mean_embedding(pb->n_src, l, d, pb->xs, pb->xf, p->sigma, ctx->wmu, st));
  HIPCHK(mean_embedding(pb->n_tgt, l, d, pb->ys, pb->yf, p->sigma, ctx->wnu, st));
  HIPCHK(mean_gram(pb->n_src, d, pb->xs, p->sigma, ctx->dsc + 0, ctx->part, st));
  HIPCHK(mean_gram(pb->n_tgt, d, pb->ys, p->sigma, ctx->dsc + 1, ctx->part, st));
  HIPCHK(build_z(l, d, pb->xf, pb->yf, ctx->wmu, ctx->wnu, p->lambda2, z, wsum, st));
  if (!dg) HIPCHK(cholesky_upper(l, ctx->Kb, 0.0, R, ctx->T1, ctx->dint, st, Linv));
  KCHK(sync_read(ctx, 2, 1));
  *q2 = ctx->hsc[0] + ctx->hsc[1];
  if (ctx->hint[0] != 0)
    return fail(ctx, KOT_ERR_FACTOR, "K + eps I is not positive definite (pivot %d)", ctx->hint[0]);
  return KOT_OK;
}

// The setup work that does not need the factor R (mean embeddings, q^2, z, KK, the default step's bounds,
// |z|^2 and the network's start), run on the second stream while the calling thread factorizes K + eps I.
// ctx: the side context; own: the calling context, whose buffers receive the results.
kot_status setup_side(kot_ctx* ctx, kot_ctx* own, const kot_problem* pb, const kot_params* p, bool predict,
                      Prelude* pre) {
  const int l = pb->l, d = pb->d;
  hipStream_t st = ctx->stream;
  HIPCHK(mean_embedding(pb->n_src, l, d, pb->xs, pb->xf, p->sigma, own->wmu, st));
  HIPCHK(mean_embedding(pb->n_tgt, l, d, pb->ys, pb->yf, p->sigma, own->wnu, st));
  HIPCHK(mean_gram(pb->n_src, d, pb->xs, p->sigma, ctx->dsc + 0, ctx->part, st));
  HIPCHK(mean_gram(pb->n_tgt, d, pb->ys, p->sigma, ctx->dsc + 1, ctx->part, st));
  HIPCHK(build_z(l, d, pb->xf, pb->yf, own->wmu, own->wnu, p->lambda2, own->zb, own->wsumb, st));
  HIPCHK(hadamard_square(l * l, own->Kb, own->KKb, st));
  HIPCHK(rowsum_abs_max(l, own->Qb, false, ctx->dsc + SL_ETA, ctx->part, st));
  HIPCHK(rowsum_abs_max(l, own->KKb, false, ctx->dsc + SL_ETA + 1, ctx->part, st));
  HIPCHK(dot(l, own->zb, own->zb, ctx->dsc + SL_ZZ, ctx->part, st));
  if (predict) {
    CoreView cv;
    cv.l = l; cv.Q = own->Qb; cv.z = own->zb; cv.wsum = own->wsumb; cv.KK = own->KKb;
    cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
    KCHK(predict_gamma0(ctx, cv, own->Kb, p->ws_F, p->ws_H, p->ws_theta, own->S[1].g));
  }
  KCHK(sync_read(ctx));
  pre->q2 = ctx->hsc[0] + ctx->hsc[1];
  pre->eta = default_eta_value(ctx->hsc[SL_ETA], ctx->hsc[SL_ETA + 1], p->lambda2);
  pre->zz = ctx->hsc[SL_ZZ];
  return KOT_OK;
}

// setup_impl with the factorization on the calling stream and setup_side beside it; the core buffers of ctx
// hold Q, z, R, w_mu + w_nu, K + eps I and KK on return (and Linv, when given, R^-T).
kot_status setup_overlapped(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, bool predict, Prelude* pre,
                            double* Linv, double* rd, bool* diag) {
  const int l = pb->l, d = pb->d;
  hipStream_t st = ctx->stream;
  KCHK(side_ensure(ctx, l, std::max(pb->n_src, pb->n_tgt)));
  HIPCHK(gram_build(l, d, pb->xf, pb->yf, p->sigma, ctx->Qb, ctx->Kb, st));
  HIPCHK(add_diag(l, p->eps_jitter, ctx->Kb, st));  // K + eps I = R^T R from here on; read-only below
  KCHK(kdiag_factor(ctx, l, p, ctx->Rb, rd, Linv, diag));
  KCHK(side_post(ctx, [ctx, pb, p, predict, pre]() { return setup_side(ctx->side->c, ctx, pb, p, predict, pre); }));
  const hipError_t e = *diag ? hipSuccess : cholesky_upper(l, ctx->Kb, 0.0, ctx->Rb, ctx->T1, ctx->dint, st, Linv);
  const kot_status rc = e != hipSuccess ? fail(ctx, KOT_ERR_HIP, "cholesky_upper: %s", hipGetErrorString(e))
                                        : sync_read(ctx);
  const kot_status rs = side_join(ctx);  // joined even when the factorization failed
  KCHK(rc);
  KCHK(rs);
  if (ctx->hint[0] != 0)
    return fail(ctx, KOT_ERR_FACTOR, "K + eps I is not positive definite (pivot %d)", ctx->hint[0]);
  return KOT_OK;
}

// Caller-supplied factors must be upper triangular (the products with R skip its zero triangle).
kot_status check_upper(kot_ctx* ctx, int l, const double* R) {
  HIPCHK(count_lower_nonzero(l, R, ctx->dint, ctx->stream));
  KCHK(sync_read(ctx, 0, 1));
  if (ctx->hint[0] != 0)
    return fail(ctx, KOT_ERR_ARG, "R must be upper triangular (%d nonzero entries below the diagonal)", ctx->hint[0]);
  return KOT_OK;
}

kot_status check_problem(kot_ctx* ctx, const kot_problem* pb) {
  if (!pb) return fail(ctx, KOT_ERR_ARG, "problem is NULL");
  if (pb->l < 1 || pb->d < 1 || pb->n_src < 1 || pb->n_tgt < 1)
    return fail(ctx, KOT_ERR_ARG, "sizes must be >= 1 (l=%d d=%d n_src=%d n_tgt=%d)", pb->l, pb->d, pb->n_src, pb->n_tgt);
  if (pb->d > 64) return fail(ctx, KOT_ERR_ARG, "d must be <= 64");
  if (pb->l > 4096) return fail(ctx, KOT_ERR_ARG, "l must be <= 4096");
  // the mean-Gram sum keeps one partial per 64 x 64 tile pair: (2^20 / 64)^2 doubles (2 GiB) at the cap
  if (pb->n_src > (1 << 20) || pb->n_tgt > (1 << 20)) return fail(ctx, KOT_ERR_ARG, "n_src and n_tgt must be <= 2^20");
  if (!pb->xs || !pb->ys || !pb->xf || !pb->yf) return fail(ctx, KOT_ERR_ARG, "null point array");
  return KOT_OK;
}

kot_status check_ctx(kot_ctx* ctx) {
  if (!ctx) return KOT_ERR_ARG;
  ctx->err.clear();
  g_prof = &ctx->prof;
  g_gemm_ws = ctx->gemm_ws;
  g_gemm_ws_cap = ctx->gemm_ws_cap;
  g_gemm_tune = ctx->tuned ? ctx->tune : nullptr;
  // the context's own stream does not order after the null stream: wait for work the caller queued there
  if (ctx->own_stream && hipStreamSynchronize(nullptr) != hipSuccess) return fail(ctx, KOT_ERR_HIP, "null stream sync");
  if (hipSetDevice(ctx->device) != hipSuccess) return fail(ctx, KOT_ERR_HIP, "hipSetDevice failed");
  return KOT_OK;
}

}  // namespace

// ================================================================================================
extern "C" {

void kot_params_default(kot_params* p) {
  if (!p) return;
  std::memset(p, 0, sizeof(*p));
  p->sigma = 1.0;
  p->lambda1 = 1e-3;
  p->lambda2 = 1e-3;
  p->eps_jitter = 1e-10;
  p->tol = 1e-6;
  p->max_iter = 200;
  p->cg_max_iter = 20;
  p->tau = 0.5;
  p->kappa = 0.5;
  p->alpha1 = 1e-6;
  p->alpha2 = 1.0;
  p->beta0 = 0.5;
  p->beta1 = 1.0 / 1.2;
  p->beta2 = 5.0;
  p->theta0 = 1.0;
  p->theta_min = 1e-6;
  p->theta_max = 1e6;
  p->eg_step = 0.0;
  p->precision = KOT_FP64;
  p->safeguard = KOT_SAFEGUARD_EG;
  p->null_step = 0;
  p->eig_max_sweeps = 30;
  p->eig_inner_sweeps = 1;
  p->closed_start = 0;
  p->kdiag_tol = 1e-12;
  p->warm_eig = 1;
  p->lift_x0 = 1;
  p->ws_F = 0;
  p->ws_H = 0;
  p->ws_theta = nullptr;
  p->overlap = 1;
  p->lowp_min_rows = 64;
  p->precond = KOT_PRECOND_NONE;
  p->schur_solver = KOT_SCHUR_CG;
}

kot_status kot_create(kot_ctx** out, int device, void* hip_stream) {
  if (!out) return KOT_ERR_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return KOT_ERR_ARG;
  kot_ctx* ctx = new kot_ctx();
  ctx->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete ctx; return KOT_ERR_HIP; }
  if (hip_stream) {
    ctx->stream = (hipStream_t)hip_stream;
  } else {
    if (hipStreamCreateWithFlags(&ctx->stream, hipStreamNonBlocking) != hipSuccess) { delete ctx; return KOT_ERR_HIP; }
    ctx->own_stream = true;
  }
  bool ok = gemm_reserve() == hipSuccess && hipMalloc(&ctx->dsc, kScalarBytes) == hipSuccess &&
            hipHostMalloc(&ctx->hsc, kScalarBytes, hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess &&
            hipHostGetDevicePointer(reinterpret_cast<void**>(&ctx->hsc_dev), ctx->hsc, 0) == hipSuccess &&
            hipEventCreate(&ctx->ev0) == hipSuccess && hipEventCreate(&ctx->ev1) == hipSuccess;
  if (ok) {
    ctx->dint = reinterpret_cast<int*>(ctx->dsc + kScalarDoubles);
    ctx->hint = reinterpret_cast<int*>(ctx->hsc + kScalarDoubles);
  }
  if (!ok) { kot_destroy(ctx); return KOT_ERR_HIP; }
  *out = ctx;
  return KOT_OK;
}

kot_status kot_destroy(kot_ctx* ctx) {
  if (!ctx) return KOT_ERR_ARG;
  hipSetDevice(ctx->device);
  if (ctx->stream) hipStreamSynchronize(ctx->stream);
  side_destroy(ctx);
  if (ctx->trtri_graph) hipGraphExecDestroy(ctx->trtri_graph);
  for (kot_ctx* ln : ctx->lanes) kot_destroy(ln);
  ctx->lanes.clear();
  free_ws(ctx);
  for (void* p : ctx->mbufs) hipFree(p);
  ctx->mbufs.clear();
  if (ctx->pot_part) hipFree(ctx->pot_part);
  hipFree(ctx->dsc);
  hipHostFree(ctx->hsc);
  if (ctx->ev0) hipEventDestroy(ctx->ev0);
  if (ctx->ev1) hipEventDestroy(ctx->ev1);
  if (ctx->own_stream && ctx->stream) hipStreamDestroy(ctx->stream);
  delete ctx;
  return KOT_OK;
}

// Message of the calling thread's last failed context-free call (kot_eigh_noalloc), else "null context".
static thread_local char g_free_err[512] = "null context";

const char* kot_last_error(const kot_ctx* ctx) { return ctx ? ctx->err.c_str() : g_free_err; }

static kot_status free_fail(kot_status st, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_free_err, sizeof(g_free_err), fmt, ap);
  va_end(ap);
  return st;
}

kot_status kot_eigh_noalloc(int device, void* hip_stream, int l, const double* Z, double* P, double* w,
                            const kot_params* p) {
  if (!Z || !P || !w || !p) return free_fail(KOT_ERR_ARG, "kot_eigh_noalloc: null argument");
  if (l < 1 || l > kNoAllocMaxL)
    return free_fail(KOT_ERR_ARG, "kot_eigh_noalloc: l = %d is outside 1..%d (the size its static scratch holds)",
                     l, kNoAllocMaxL);
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return free_fail(KOT_ERR_ARG, "kot_eigh_noalloc: no HIP device %d", device);
  int prev = 0;
  if (hipGetDevice(&prev) != hipSuccess) return free_fail(KOT_ERR_HIP, "kot_eigh_noalloc: hipGetDevice failed");
  if (hipSetDevice(device) != hipSuccess) return free_fail(KOT_ERR_HIP, "kot_eigh_noalloc: hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int max_sw = p->eig_max_sweeps > 0 ? p->eig_max_sweeps : 30;
  const int inner = p->eig_inner_sweeps > 0 ? p->eig_inner_sweeps : 1;
  int sw = 0;
  double rel = 0.0;
  hipError_t e = eigh_jacobi_noalloc(device, l, Z, P, w, max_sw, inner, 1e-14, &sw, &rel, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  (void)hipSetDevice(prev);
  if (e != hipSuccess) return free_fail(KOT_ERR_HIP, "kot_eigh_noalloc: %s", hipGetErrorString(e));
  if (!(rel <= 1e-14)) {
    if (!std::isfinite(rel)) return free_fail(KOT_ERR_NUMERIC, "kot_eigh_noalloc: non-finite matrix");
    return free_fail(KOT_ERR_EIG, "kot_eigh_noalloc: Jacobi did not converge in %d sweeps (off/norm = %.3e)", sw, rel);
  }
  return KOT_OK;
}

kot_status kot_setup(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, double* Q, double* z, double* R,
                     double* wsum, double* q2) {
  KCHK(check_ctx(ctx));
  KCHK(check_problem(ctx, pb));
  KCHK(check_params(ctx, p, true));
  if (!Q || !z || !R || !wsum || !q2) return fail(ctx, KOT_ERR_ARG, "null output");
  KCHK(ensure_ws(ctx, pb->l, std::max(pb->n_src, pb->n_tgt)));
  return setup_impl(ctx, pb, p, Q, z, R, wsum, q2, nullptr, ctx->rdb);
}

kot_status kot_solve(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, const double* gamma0, kot_result* res) {
  KCHK(check_ctx(ctx));
  KCHK(check_problem(ctx, pb));
  KCHK(check_params(ctx, p, true));
  if (!res || !res->gamma) return fail(ctx, KOT_ERR_ARG, "result or result->gamma is NULL");
  KCHK(ensure_ws(ctx, pb->l, std::max(pb->n_src, pb->n_tgt)));
  CoreView cv;
  cv.l = pb->l; cv.Q = ctx->Qb; cv.z = ctx->zb; cv.R = ctx->Rb; cv.wsum = ctx->wsumb;
  cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  // the lifted start needs R^-T: the factorization forms it beside R (the buffer is free until the first
  // extragradient step)
  double* Linv = (gamma0 || p->ws_theta || p->closed_start == 1) && p->lift_x0 ? ctx->Xh : nullptr;
  cv.Linv = Linv;
  bool diag = false;
  if (overlap_ok(ctx, p, pb->l)) {
    Prelude pre;
    KCHK(setup_overlapped(ctx, pb, p, p->ws_theta && !gamma0, &pre, Linv, ctx->rdb, &diag));
    cv.q2 = pre.q2;
    cv.kb_state = 2;
    cv.KK = ctx->KKb;
    cv.rd = diag ? ctx->rdb : nullptr;
    const kot_status s = run_alg2(ctx, cv, p, gamma0, res, &pre);
    res->kdiag = diag ? 1 : 0;
    return s;
  }
  double q2 = 0.0;
  KCHK(setup_impl(ctx, pb, p, ctx->Qb, ctx->zb, ctx->Rb, ctx->wsumb, &q2, Linv, ctx->rdb, &diag));
  cv.q2 = q2;
  cv.kb_state = 1;
  cv.rd = diag ? ctx->rdb : nullptr;
  const kot_status s = run_alg2(ctx, cv, p, gamma0, res);
  res->kdiag = diag ? 1 : 0;
  return s;
}

kot_status kot_solve_core(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, double q2,
                          const double* wsum, const kot_params* p, const double* gamma0, kot_result* res) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096) return fail(ctx, KOT_ERR_ARG, "l must be in [1, 4096]");
  if (!Q || !z || !R || !wsum || !res || !res->gamma) return fail(ctx, KOT_ERR_ARG, "null pointer argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.wsum = wsum; cv.q2 = q2; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  return run_alg2(ctx, cv, p, gamma0, res);
}

kot_status kot_eigh(kot_ctx* ctx, int l, const double* Z, double* P, double* w, const kot_params* p) {
  KCHK(check_ctx(ctx));
  if (l < 1 || l > 4096 || !Z || !P || !w || !p) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  HIPCHK(form_z(l, Z, 0.0, Z, 0.0, ctx->Z, ctx->stream));  // (Z + Z^T)/2
  int sw = 0, npos = 0;
  kot_status s = eig_run(ctx, l, ctx->Z, nullptr, P, w, p, &sw, &npos);
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return s;
}

kot_status kot_residual(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, const double* gamma,
                        const double* X, const kot_params* p, double* r1, double* r2, double* norms) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096 || !Q || !z || !R || !gamma || !X || !r1 || !r2 || !norms)
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  State& s = ctx->S[3];
  HIPCHK(vec_copy(l, gamma, s.g, ctx->stream));
  HIPCHK(vec_copy(l * l, X, s.X, ctx->stream));
  KCHK(residual_state(ctx, cv, s, nullptr, p, nullptr));
  HIPCHK(vec_copy(l, s.r1, r1, ctx->stream));
  HIPCHK(vec_copy(l * l, s.r2, r2, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  norms[0] = s.r1n;
  norms[1] = s.r2n;
  norms[2] = (double)s.a;
  return KOT_OK;
}

kot_status kot_ssn_direction(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, const double* gamma,
                             const double* X, double mu, const kot_params* p, double* dgamma, double* dX, double* info) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096 || !Q || !z || !R || !gamma || !X || !dgamma || !dX || !info || !(mu > 0.0))
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  KCHK(prepare_core(ctx, cv));
  State& s = ctx->S[0];
  HIPCHK(vec_copy(l, gamma, s.g, ctx->stream));
  HIPCHK(vec_copy(l * l, X, s.X, ctx->stream));
  KCHK(residual_state(ctx, cv, s, nullptr, p, nullptr));
  DirInfo di;
  KCHK(ssn_direction(ctx, cv, s, mu, p, &di));
  HIPCHK(vec_copy(l, ctx->dg, dgamma, ctx->stream));
  HIPCHK(vec_copy(l * l, ctx->dX, dX, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  info[0] = di.cg_iters;
  info[1] = di.cg_res;
  info[2] = s.a;
  info[3] = s.rn;
  return KOT_OK;
}

kot_status kot_schur_matvec(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R,
                            const double* gamma, const double* X, double mu, const kot_params* p, int reps,
                            const double* v, double* y, double* info) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096 || !Q || !z || !R || !gamma || !X || !v || !y || !info || !(mu > 0.0) || reps < 1)
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  KCHK(prepare_core(ctx, cv));
  State& s = ctx->S[0];
  HIPCHK(vec_copy(l, gamma, s.g, ctx->stream));
  HIPCHK(vec_copy(l * l, X, s.X, ctx->stream));
  KCHK(residual_state(ctx, cv, s, nullptr, p, nullptr));
  hipStream_t st = ctx->stream;
  TPlan tp = make_tplan(l, s.a, mu, s.P, s.s);
  HIPCHK(mm(st, 1, 0, l, l, l, 1.0, s.P, l, nullptr, cv.R, l, 0.0, ctx->Bm, l, TRI_B_UPPER));
  const int mode = p->precision == KOT_MIXED_BF16 ? 1 : (p->precision == KOT_MIXED_BF16X3 ? 2 : 0);
  if (p->precision != KOT_FP64) {
    HIPCHK(f64_to_f32((long long)l * l, ctx->Bm, ctx->Bf, st));
    if (mode != 0)
      HIPCHK(chain_prep(l, chain_ldp(l), ctx->Bm, ctx->Bh, ctx->BhT, mode == 2 ? ctx->Bl : nullptr,
                        mode == 2 ? ctx->BlT : nullptr, st));
  }
  HIPCHK(hipEventRecord(ctx->ev0, st));
  for (int r = 0; r < reps; ++r) {
    if (p->precision == KOT_FP64) KCHK(schur_matvec(ctx, cv, tp, v, y));
    else KCHK(schur_matvec_lowp(ctx, cv, tp, v, y, mode));
  }
  HIPCHK(hipEventRecord(ctx->ev1, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  info[0] = s.a;
  info[1] = tp.m;
  info[2] = tp.comp ? 1.0 : 0.0;
  info[3] = ms / reps;
  return KOT_OK;
}

kot_status kot_eg_step(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, const double* gamma,
                       const double* X, double eta, const kot_params* p, double* gamma_out, double* X_out) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096 || !Q || !z || !R || !gamma || !X || !gamma_out || !X_out || !(eta > 0.0))
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  KCHK(r1_op(ctx, cv, gamma, X, ctx->vtmp));
  KCHK(eg_step_impl(ctx, cv, gamma, X, ctx->vtmp, eta, gamma_out, X_out, false, p, nullptr));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_cholesky(kot_ctx* ctx, int l, const double* A, double eps, double* R, double* Rit) {
  KCHK(check_ctx(ctx));
  if (l < 1 || l > 4096 || !A || !R || !(eps >= 0.0)) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  HIPCHK(cholesky_upper(l, A, eps, R, ctx->T1, ctx->dint, ctx->stream, Rit));
  KCHK(sync_read(ctx, 0, 1));
  if (ctx->hint[0] != 0) return fail(ctx, KOT_ERR_FACTOR, "matrix is not positive definite (pivot %d)", ctx->hint[0]);
  return KOT_OK;
}

kot_status kot_solve_batched(kot_ctx* ctx, int nprob, const kot_problem* probs, const kot_params* prms, int nparams,
                             const double* const* gamma0, kot_result* results, int* status, int lanes) {
  KCHK(check_ctx(ctx));
  if (nprob < 0 || (nprob > 0 && (!probs || !prms || !results || !status)) || (nparams != 1 && nparams != nprob))
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  for (int i = 0; i < nprob; ++i) {
    KCHK(check_problem(ctx, &probs[i]));
    KCHK(check_params(ctx, &prms[nparams == 1 ? 0 : i], true));
    if (!results[i].gamma) return fail(ctx, KOT_ERR_ARG, "results[%d].gamma is NULL", i);
  }
  if (nprob == 0) return KOT_OK;
  if (lanes <= 0) lanes = 8;  // more lanes than hardware queues: a lane waiting on the host leaves room to others
  lanes = std::min(lanes, std::min(nprob, 16));
  while ((int)ctx->lanes.size() < lanes) {
    kot_ctx* c = nullptr;
    kot_status s = kot_create(&c, ctx->device, nullptr);
    if (s != KOT_OK) return fail(ctx, s, "could not create a batch lane");
    c->is_lane = true;
    ctx->lanes.push_back(c);
  }
  // inputs may come from any stream of the caller: make them visible to the lanes' streams
  HIPCHK(hipDeviceSynchronize());
  std::atomic<int> next(0);
  auto worker = [&](kot_ctx* lane) {
    for (;;) {
      const int i = next.fetch_add(1);
      if (i >= nprob) break;
      const kot_params* p = &prms[nparams == 1 ? 0 : i];
      status[i] = kot_solve(lane, &probs[i], p, gamma0 ? gamma0[i] : nullptr, &results[i]);
    }
  };
  std::vector<std::thread> th;
  for (int t = 0; t < lanes; ++t) {
    if (ctx->tuned) {
      std::copy(ctx->tune, ctx->tune + kTuneBuckets, ctx->lanes[t]->tune);
      ctx->lanes[t]->tuned = true;
    }
    th.emplace_back(worker, ctx->lanes[t]);
  }
  for (auto& t : th) t.join();
  g_prof = &ctx->prof;
  g_gemm_ws = ctx->gemm_ws;
  g_gemm_ws_cap = ctx->gemm_ws_cap;
  int worst = KOT_OK;
  for (int i = 0; i < nprob; ++i)
    if (status[i] < worst) worst = status[i];
  if (worst < 0) {
    for (int i = 0; i < nprob; ++i)
      if (status[i] == worst) return fail(ctx, (kot_status)worst, "problem %d failed with status %d", i, worst);
  }
  return KOT_OK;
}

kot_status kot_autotune(kot_ctx* ctx, const int* sizes, int nsizes, const char* path, int* table_out) {
  KCHK(check_ctx(ctx));
  if (nsizes < 1 || !sizes) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  int Lmax = 1;
  for (int i = 0; i < nsizes; ++i) {
    if (sizes[i] < 1 || sizes[i] > 4096) return fail(ctx, KOT_ERR_ARG, "sizes must be in [1, 4096]");
    Lmax = std::max(Lmax, sizes[i]);
  }
  KCHK(ensure_ws(ctx, Lmax, 0));
  if (!ctx->tuned) {
    for (int b = 0; b < kTuneBuckets; ++b) ctx->tune[b] = 256;
  }
  hipStream_t st = ctx->stream;
  double* A = ctx->T1;
  double* B = ctx->T2;
  double* Cm = ctx->T3;
  HIPCHK(vec_fill(Lmax * Lmax, 0.5, A, st));
  HIPCHK(vec_fill(Lmax * Lmax, 0.25, B, st));
  HIPCHK(vec_fill(Lmax, 1.0, ctx->vtmp, st));
  const int cand[5] = {0, 128, 256, 512, 1024};
  int local[kTuneBuckets];
  std::copy(ctx->tune, ctx->tune + kTuneBuckets, local);
  for (int i = 0; i < nsizes; ++i) {
    const int L = sizes[i];
    double best_t = 1e300;
    int best = 256;
    for (int c : cand) {
      local[gemm_tune_bucket(L)] = c;
      g_gemm_tune = local;
      for (int rep = 0; rep < 2; ++rep) {  // warm, then timed
        HIPCHK(hipEventRecord(ctx->ev0, st));
        for (int r = 0; r < 5; ++r) {
          HIPCHK(mm(st, 0, 0, L, L, L, 1.0, A, L, nullptr, B, L, 0.0, Cm, L));
          HIPCHK(mm(st, 0, 1, std::max(1, L / 2), L, L, 1.0, A, L, ctx->vtmp, B, L, 0.0, Cm, L));
        }
        HIPCHK(hipEventRecord(ctx->ev1, st));
        HIPCHK(hipEventSynchronize(ctx->ev1));
      }
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
      if (ms < best_t) { best_t = ms; best = c; }
    }
    local[gemm_tune_bucket(L)] = best;
  }
  std::copy(local, local + kTuneBuckets, ctx->tune);
  ctx->tuned = true;
  g_gemm_tune = ctx->tune;
  if (table_out) std::copy(ctx->tune, ctx->tune + kTuneBuckets, table_out);
  if (path) {
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(ctx, KOT_ERR_ARG, "cannot write %s", path);
    std::fprintf(f, "kot-gemm-tune 1\n");
    for (int b = 0; b < kTuneBuckets; ++b) std::fprintf(f, "%d %d\n", b, ctx->tune[b]);
    std::fclose(f);
  }
  return KOT_OK;
}

kot_status kot_autotune_load(kot_ctx* ctx, const char* path) {
  KCHK(check_ctx(ctx));
  if (!path) return fail(ctx, KOT_ERR_ARG, "path is NULL");
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, KOT_ERR_ARG, "cannot read %s", path);
  int ver = 0;
  int tab[kTuneBuckets];
  for (int b = 0; b < kTuneBuckets; ++b) tab[b] = 256;
  if (std::fscanf(f, "kot-gemm-tune %d", &ver) != 1 || ver != 1) {
    std::fclose(f);
    return fail(ctx, KOT_ERR_ARG, "%s is not a tuning table", path);
  }
  int b = 0, v = 0;
  while (std::fscanf(f, "%d %d", &b, &v) == 2)
    if (b >= 0 && b < kTuneBuckets && v >= 0 && v <= 4096) tab[b] = v;
  std::fclose(f);
  std::copy(tab, tab + kTuneBuckets, ctx->tune);
  ctx->tuned = true;
  g_gemm_tune = ctx->tune;
  return KOT_OK;
}

int kot_mlp_params(int F, int H) { return F * H + H + H * H + H + H + 1; }

kot_status kot_features(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, const double* wsum,
                        double q2, const kot_params* p, float* X) {
  KCHK(check_ctx(ctx));
  KCHK(check_params(ctx, p, false));
  if (l < 1 || l > 4096 || !Q || !z || !R || !wsum || !X) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, l, 0));
  KCHK(check_upper(ctx, l, R));
  KCHK(ensure_mlp(ctx, l, 1, l));
  CoreView cv;
  cv.l = l; cv.Q = Q; cv.z = z; cv.R = R; cv.wsum = wsum; cv.q2 = q2; cv.lam1 = p->lambda1; cv.lam2 = p->lambda2;
  KCHK(prepare_core(ctx, cv));
  HIPCHK(features(l, Q, z, wsum, ctx->Kb, cv.KK, cv.lam1, ctx->rs3, ctx->dsc + SL_POOL, X, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_mlp_forward(kot_ctx* ctx, int n, int F, int H, const float* X, const float* theta, float* out) {
  KCHK(check_ctx(ctx));
  if (n < 1 || F < 1 || H < 1 || !X || !theta || !out) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_mlp(ctx, n, H, 1));
  KCHK(mlp_forward_impl(ctx, n, mlp_view(F, H, theta), X, out));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_mlp_loss_grad(kot_ctx* ctx, int n, int F, int H, const float* X, const float* y, const float* theta,
                             float* grad, double* loss) {
  KCHK(check_ctx(ctx));
  if (n < 1 || F < 1 || H < 1 || !X || !y || !theta || !grad || !loss) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  if (!ctx->dsc) return fail(ctx, KOT_ERR_ARG, "context not initialised");
  KCHK(ensure_ws(ctx, 1, 0));  // reduction partials
  KCHK(ensure_mlp(ctx, n, H, 1));
  return mlp_loss_grad_impl(ctx, n, mlp_view(F, H, theta), X, y, grad, loss);
}

kot_status kot_mlp_adam(kot_ctx* ctx, int P, float* theta, const float* grad, float* m, float* v, int t, float lr,
                        float beta1, float beta2, float eps) {
  KCHK(check_ctx(ctx));
  if (P < 1 || t < 1 || !theta || !grad || !m || !v) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  HIPCHK(adam_f32(P, theta, grad, m, v, lr, beta1, beta2, eps, t, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_warmstart(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, int F, int H, const float* theta,
                         double* gamma0) {
  KCHK(check_ctx(ctx));
  KCHK(check_problem(ctx, pb));
  KCHK(check_params(ctx, p, true));
  if (!theta || !gamma0 || H < 1) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  KCHK(ensure_ws(ctx, pb->l, std::max(pb->n_src, pb->n_tgt)));
  double q2 = 0.0;
  KCHK(setup_impl(ctx, pb, p, ctx->Qb, ctx->zb, ctx->Rb, ctx->wsumb, &q2));
  CoreView cv;
  cv.l = pb->l; cv.Q = ctx->Qb; cv.z = ctx->zb; cv.R = ctx->Rb; cv.wsum = ctx->wsumb; cv.q2 = q2;
  cv.lam1 = p->lambda1; cv.lam2 = p->lambda2; cv.kb_state = 1;
  KCHK(prepare_core(ctx, cv));
  KCHK(predict_gamma0(ctx, cv, ctx->Kb, F, H, theta, gamma0));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_potentials(kot_ctx* ctx, const kot_problem* pb, const kot_params* p, const double* gamma, int m,
                          const double* xq, const double* yq, double* u, double* v, double* Tx) {
  KCHK(check_ctx(ctx));
  KCHK(check_problem(ctx, pb));
  KCHK(check_params(ctx, p, true));
  if (m < 0 || !gamma || (m > 0 && !((xq && u) || (yq && v))) || (Tx && !xq))
    return fail(ctx, KOT_ERR_ARG, "invalid argument");
  if (m == 0) return KOT_OK;
  const int d = pb->d;
  const int splits_x = potential_splits(m, pb->n_src, pb->l), splits_y = potential_splits(m, pb->n_tgt, pb->l);
  const size_t need = std::max(potential_part_size(m, d, splits_x), potential_part_size(m, d, splits_y));
  if (need > ctx->pot_part_cap) {
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (ctx->pot_part) hipFree(ctx->pot_part);
    ctx->pot_part = nullptr;
    ctx->pot_part_cap = 0;
    if (hipMalloc(&ctx->pot_part, need * sizeof(double)) != hipSuccess) {
      ctx->pot_part = nullptr;
      return fail(ctx, KOT_ERR_OOM, "potential workspace allocation failed");
    }
    ctx->pot_part_cap = need;
  }
  if (xq && u)
    HIPCHK(potential_eval(m, d, xq, pb->xs, pb->n_src, pb->xf, pb->l, gamma, p->sigma, p->lambda2, splits_x,
                          ctx->pot_part, u, Tx, ctx->stream));
  if (yq && v)
    HIPCHK(potential_eval(m, d, yq, pb->ys, pb->n_tgt, pb->yf, pb->l, gamma, p->sigma, p->lambda2, splits_y,
                          ctx->pot_part, v, nullptr, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

kot_status kot_profile(kot_ctx* ctx, int enable, double* out, int nclass) {
  KCHK(check_ctx(ctx));
  // launches of the second and third streams count with the context's own
  Profiler* side = ctx->side ? &ctx->side->c->prof : nullptr;
  Profiler* side2 = ctx->side2 ? &ctx->side2->c->prof : nullptr;
  if (enable) {
    ctx->prof.clear();
    ctx->prof.on = true;
    if (side) side->clear();
    if (side2) side2->clear();
    return KOT_OK;
  }
  ctx->prof.on = false;
  HIPCHK(hipStreamSynchronize(ctx->stream));
  for (SideRunner* s : {ctx->side, ctx->side2}) {
    if (!s) continue;
    s->c->prof.on = false;
    HIPCHK(hipStreamSynchronize(s->c->stream));
  }
  if (out) {
    for (int c = 0; c < nclass * 4; ++c) out[c] = 0.0;
    for (const Profiler* pf : {(const Profiler*)&ctx->prof, (const Profiler*)side, (const Profiler*)side2}) {
      if (!pf) continue;
      for (const auto& r : pf->recs) {
        if (r.cls >= nclass || !r.a || !r.b) continue;
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        out[4 * r.cls + 0] += 1.0;
        out[4 * r.cls + 1] += ms;
        out[4 * r.cls + 2] += r.flops;
        out[4 * r.cls + 3] += r.bytes;
      }
    }
  }
  ctx->prof.clear();
  if (side) side->clear();
  if (side2) side2->clear();
  return KOT_OK;
}

kot_status kot_gemm(kot_ctx* ctx, int transa, int transb, int m, int n, int k, double alpha, const double* A, int lda,
                    const double* s, const double* B, int ldb, double beta, double* C, int ldc, int tri, int sym) {
  KCHK(check_ctx(ctx));
  if (m < 0 || n < 0 || k < 1 || !A || !B || !C) return fail(ctx, KOT_ERR_ARG, "invalid argument");
  if (tri < 0 || tri > 15 || (tri & 3) == 3 || (tri & 12) == 12 || (sym && m != n))
    return fail(ctx, KOT_ERR_ARG, "invalid tri / sym");
  if (std::max(m, n) <= 4096) KCHK(ensure_ws(ctx, std::max(std::max(m, n), 1), 0));  // split-K workspace
  HIPCHK(mm(ctx->stream, transa ? 1 : 0, transb ? 1 : 0, m, n, k, alpha, A, lda, s, B, ldb, beta, C, ldc, tri,
            sym != 0));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return KOT_OK;
}

}  // extern "C"
