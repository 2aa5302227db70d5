/*
 * kotssn — semismooth Newton (SSN) solver for the kernel-based optimal-transport estimator of
 * Lin, Cuturi & Jordan, "A Specialized Semismooth Newton Method for Kernel-Based Optimal Transport" (2023),
 * on one AMD Instinct MI355X (gfx950).
 *
 * Conventions for every entry point:
 *  - Array arguments named in a "device" comment are device pointers (HIP memory on the context's device);
 *    arrays named "host" are host pointers.  Matrices are row-major, FP64, leading dimension = number of
 *    columns (l for l x l matrices, d for point sets), contiguous.
 *  - The caller owns every input and output buffer.  The library owns the context's workspace, which it
 *    sizes lazily from the largest l it has seen and frees in kot_destroy.
 *  - All work is enqueued on the context's stream; every call returns after that stream has drained, so
 *    outputs are ready on return.
 *  - Errors are returned as kot_status; a message for the last error of a context is available from
 *    kot_last_error.  Nothing throws across this boundary.  Inputs are validated before any kernel is
 *    launched: l, n, d >= 1, sigma, lambda1, lambda2 > 0, pointers non-null (KOT_ERR_ARG otherwise).
 *  - Not thread-safe per context: calls that share a context must not overlap.
 */
#ifndef KOTSSN_H
#define KOTSSN_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kot_ctx kot_ctx;

typedef enum {
  KOT_OK = 0,
  KOT_NOT_CONVERGED = 1,   /* outputs valid; tolerance not met within max_iter */
  KOT_ERR_ARG = -1,        /* invalid argument; nothing was launched */
  KOT_ERR_HIP = -2,        /* HIP runtime error */
  KOT_ERR_OOM = -3,        /* workspace allocation failed */
  KOT_ERR_FACTOR = -4,     /* K + eps I is not numerically positive definite */
  KOT_ERR_NUMERIC = -5,    /* NaN/Inf in the residual, or in a matrix given to the eigensolver */
  KOT_ERR_EIG = -6         /* eigensolver did not reach its off-diagonal tolerance */
} kot_status;

/* Arithmetic of the CG matvec chain: FP64; FP32 products; BF16 products; or split BF16 products (each FP32
 * operand x = hi + lo with hi = bf16(x), lo = bf16(x - hi), product hi*hi + hi*lo + lo*hi), all three with
 * FP32 accumulation inside FP64 iterative refinement. */
typedef enum { KOT_FP64 = 0, KOT_FP32 = 1, KOT_MIXED_BF16 = 2, KOT_MIXED_BF16X3 = 3 } kot_precision;
/* Algorithm 2 with its extragradient safeguard (EG), the regularized SSN steps alone (NONE), or the safeguard
 * alone: pure extragradient iterations on Eq. (4.1), the comparison method of Appendix F (EG_ONLY). */
typedef enum { KOT_SAFEGUARD_EG = 0, KOT_SAFEGUARD_NONE = 1, KOT_SAFEGUARD_EG_ONLY = 2 } kot_safeguard;
/* CG on the Schur system of Algorithm 1 as the paper runs it (NONE), or preconditioned with the inverse of the
 * system's diagonal (JACOBI; not in the paper, which runs plain CG):
 * M_ii = Q_ii/(2 lambda2) + mu + [(B o B)^T Psi (B o B)]_ii with B = P^T R.  Eq. (4.5) is checked on the
 * unpreconditioned residual either way. */
typedef enum { KOT_PRECOND_NONE = 0, KOT_PRECOND_JACOBI = 1 } kot_precond;
/* Solver of that Schur system: conjugate gradients (the paper's choice) or symmetric QMR (Freund and
 * Nachtigal's simplified QMR, the other Krylov method Section 4.3 names), with the same preconditioner choice,
 * iteration cap and Eq. (4.5) test (on the true residual b - M x). */
typedef enum { KOT_SCHUR_CG = 0, KOT_SCHUR_SQMR = 1 } kot_schur_solver;

/* Parameters of Algorithm 2 and the inexactness rule Eq. (4.5).  kot_params_default fills the values
 * used throughout: tol 1e-6, max_iter 200, cg_max_iter 20 (Remark 4.5), tau = kappa = 0.5,
 * alpha1 = 1e-6, alpha2 = 1, beta0 = 0.5, beta1 = 1/1.2, beta2 = 5 (Section 5 constants, with beta1 < 1
 * as Algorithm 2's input requires; Section 5 prints 1.2, which set here runs the printed value),
 * theta0 = 1, theta in [1e-6, 1e6], eg_step = 0 (=> 0.5 / Lhat with
 * Lhat = |Q|_inf/(2 lambda2) + sqrt(|K o K|_inf)), null_step = 0 (Algorithm 2's accept test as printed:
 * w_{k+1} = SSN trial if |R(trial)| <= |R(v_{k+1})|, else v_{k+1}; 1 = opt-in variant that keeps w_k when
 * the trial is worse than w_k and w_k beats v_{k+1}), eps_jitter = 1e-10 (R^T R = K + eps I). */
typedef struct kot_params {
  double sigma;        /* Gaussian bandwidth: k(a,b) = exp(-|a-b|^2 / (2 sigma^2)) */
  double lambda1;      /* trace penalty (Eq. 3.2) */
  double lambda2;      /* RKHS-norm penalty (Eq. 3.2) */
  double eps_jitter;
  double tol;          /* stop when |r1|_2 + |r2|_F <= tol */
  int max_iter;
  int cg_max_iter;
  double tau, kappa;
  double alpha1, alpha2, beta0, beta1, beta2;
  double theta0, theta_min, theta_max;
  double eg_step;
  int precision;       /* kot_precision of the CG matvec chain (Algorithm 1): FP64, or FP32 / BF16 products with
                          FP32 accumulation inside FP64 iterative refinement (Eq. 4.5 checked in FP64) */
  int safeguard;       /* kot_safeguard */
  int null_step;
  int eig_max_sweeps;  /* Jacobi sweep cap (default 30) */
  int warm_eig;        /* 1: start each eigendecomposition from the previous eigenbasis (default 1) */
  int lift_x0;         /* with a start gamma0: 1 (default) = X0 = R^-T diag(y) R^-1 with y_i = (Q gamma0 - z)_i/(2 lambda2)
                          on constraints predicted active (gamma0_i <= -0.9 lambda1, y_i > 0), entries below
                          0.02 x the mean positive y_i set to 0; 0 = X0 = 0 */
  int ws_F, ws_H;      /* warm-start network sizes (features, width) when ws_theta is set */
  const float* ws_theta; /* device, kot_mlp layout; non-NULL: kot_solve predicts gamma0 with the network */
  int overlap;         /* 1 (default), for l >= 128: a second stream driven by a second host thread runs the
                          setup work that does not need R (mean embeddings, q^2, z, the network's start) while
                          the Cholesky factorization runs, and, with safeguard EG, the extragradient branch of
                          each iteration (its step and the residual at v_{k+1}) while the Newton direction and
                          the trial residual run.  Results are those of 0 (one stream), bit for bit.  Not used
                          by kot_solve_batched lanes. */
  int lowp_min_rows;   /* with a reduced precision: the Newton direction runs the reduced-precision chain and
                          iterative refinement only when the chain has at least this many eigen-rows
                          (min(|alpha|, l - |alpha|)); below it the chain's products are too small to gain from
                          lower precision and the FP64 CG runs instead (default 64; 0 = always) */
  int precond;         /* kot_precond of the Schur-system solver (default KOT_PRECOND_NONE) */
  int schur_solver;    /* a kot_schur_solver value; default KOT_SCHUR_CG */
  int eig_inner_sweeps; /* cap on the cyclic Jacobi sweeps a 16x16 block-pair subproblem gets per visit of the
                           eigensolver (default 1; a visit also ends after a sweep that rotated nothing) */
  int closed_start;    /* the closed-form start gamma0_i = max(z_i / Q_ii, -lambda1), the minimizer of Eq. (3.4)
                          for diagonal Q and orthogonal R (the LMI is then the box gamma >= -lambda1), lifted and
                          kept or dropped like any start: 1 = the start when neither gamma0 nor ws_theta is given;
                          2 = the replacement of a start (gamma0 or the network's) that fails the fallback test,
                          itself kept only if it passes that test; 0 (default) = not used.  Other values are
                          rejected with KOT_ERR_ARG. */
  double kdiag_tol;    /* sparsity of K (Remark 4.5): when every off-diagonal entry of K + eps I is at most kdiag_tol
                          times its largest diagonal entry, the setup drops them, so R = diag(sqrt(K_ii + eps))
                          without the factorization, and the solve's products with R (Phi, Phi*, P^T R, the
                          lifted start) become diagonal scalings (default 1e-12; 0 = always factor) */
} kot_params;

/* Samples and filling points (Section 3).  All four arrays are device pointers, row-major:
 * xs n_src x d, ys n_tgt x d, xf l x d, yf l x d.  Accepted sizes: 1 <= l <= 4096, 1 <= d <= 64,
 * 1 <= n_src, n_tgt <= 2^20; others are rejected with KOT_ERR_ARG before any launch. */
typedef struct kot_problem {
  int n_src, n_tgt, d, l;
  const double* xs;
  const double* ys;
  const double* xf;
  const double* yf;
} kot_problem;

/* Solver outputs.  gamma (device, length l) receives the dual vector; X (device, l x l, may be NULL)
 * receives the PSD multiplier; res_hist / res_v_hist (host, hist_cap entries each, may be NULL) receive
 * |R(w_k)| and |R(v_k)| for k = 0..iters, where an iteration whose accept test was decided by the lower bound
 * |R(v_k)| >= |r1(v_k)| (the trial's residual below it, so Z at v_k was not decomposed) records |r1(v_k)|; the
 * scalars are filled on return. */
typedef struct kot_result {
  double* gamma;
  double* X;
  double* res_hist;
  double* res_v_hist;
  int hist_cap;
  double ot;           /* estimator: (q2 - gamma^T (w_mu + w_nu)) / (2 lambda2), Section 3 */
  double residual;     /* |R(w)| at the returned iterate */
  int iters;           /* outer iterations performed */
  int cg_iters_total;
  int eg_accepts;      /* iterations whose w_{k+1} is the extragradient iterate */
  int null_steps;      /* iterations that kept w_k */
  int eig_sweeps_total;
  int alpha_last;      /* number of positive eigenvalues of Z at the returned iterate */
  int warm_used;       /* 1 if the start from gamma0 (given or the network's) was kept (it had |R(w0)| <= |R(0,0)|),
                          2 if it was not and the closed-form start replacing it was (closed_start = 2), else 0 */
  int lowp_directions; /* Newton directions computed with the reduced-precision chain (see lowp_min_rows) */
  double time_ms;      /* wall time of the solve on the device stream */
  int kdiag;           /* 1 if the setup took K as diagonal (kdiag_tol), else 0 */
} kot_result;

/* Fills *p with the defaults listed above (sigma, lambda1, lambda2 set to 1, 1e-3, 1e-3). */
void kot_params_default(kot_params* p);

/* Creates a context on HIP device `device`.  `hip_stream` is a hipStream_t (NULL = the context creates and
 * owns its own stream); the caller keeps ownership of a stream it passes in. */
kot_status kot_create(kot_ctx** out, int device, void* hip_stream);
kot_status kot_destroy(kot_ctx* ctx);
/* Message of the last error on this context ("" if none).  Valid until the next call on the context. */
const char* kot_last_error(const kot_ctx* ctx);

/* Dual data of Eq. (3.4) (Section 3): Q = K_X + K_Y (l x l), z (l), the upper-triangular factor R with
 * R^T R = K + eps I where K = K_X o K_Y (l x l), wsum = w_mu + w_nu at the filling points (l), and q2
 * (host scalar).  Q, z, R, wsum are device pointers; R's strictly lower triangle is written as 0.  When
 * K + eps I is diagonal to prm->kdiag_tol, its off-diagonal entries are dropped and R = diag(sqrt(K_ii + eps)).
 * Returns KOT_ERR_FACTOR if the Cholesky factorization meets a non-positive pivot. */
kot_status kot_setup(kot_ctx* ctx, const kot_problem* prob, const kot_params* prm,
                     double* Q, double* z, double* R, double* wsum, double* q2);

/* Full solve: setup (as kot_setup) then Algorithm 2 from a start w0 = (gamma0, X0): gamma0 (device, length
 * l) if given, else the network's prediction when prm->ws_theta is set, else the closed-form start when
 * prm->closed_start = 1, else the cold start (0, 0); X0 lifted from gamma0 (lift_x0) or 0.  A start is kept
 * only if |R(w0)| <= |R(0, 0)| (the fallback test); a given or predicted start that fails it is replaced by
 * the closed-form start when prm->closed_start = 2 (if that passes), else by (0, 0); res->warm_used says which. */
kot_status kot_solve(kot_ctx* ctx, const kot_problem* prob, const kot_params* prm, const double* gamma0,
                     kot_result* res);

/* Many independent problems (any mix of n_src, n_tgt, d, l): each is solved as by kot_solve.  prms holds
 * 1 entry (shared) or nprob entries; gamma0 (host array of nprob device pointers) may be NULL; results[i]
 * (gamma required) and status[i] (host) receive problem i's outputs.  The problems are spread over `lanes`
 * child contexts (0 = 8), each with its own HIP stream and workspace and driven by its own host thread, so
 * kernels of different problems overlap on the device.  Returns the most severe error status if a problem
 * failed (KOT_NOT_CONVERGED is reported per problem only). */
kot_status kot_solve_batched(kot_ctx* ctx, int nprob, const kot_problem* probs, const kot_params* prms, int nparams,
                             const double* const* gamma0, kot_result* results, int* status, int lanes);

/* GEMM tiling autotuner (not in the paper).  For each size L in sizes (host, nsizes entries, 1..4096) times the
 * two product shapes of a solve (L x L x L and L/2 x L x L with a diagonal scale) for each split-K target
 * (0 = no K split, 128, 256, 512, 1024 workgroups; default 256, doubled for triangular operands) and keeps
 * the fastest per size bucket (128-wide).  The table
 * (33 entries, copied to table_out when non-NULL) is used by every later call on this context and its batch
 * lanes; path (may be NULL) receives it as text.  kot_autotune_load installs a saved table. */
kot_status kot_autotune(kot_ctx* ctx, const int* sizes, int nsizes, const char* path, int* table_out);
kot_status kot_autotune_load(kot_ctx* ctx, const char* path);

/* Algorithm 2 on given dual data (Eq. 3.4): Q, z, R (the upper-triangular factor with R^T R = K, as
 * kot_setup / kot_cholesky return it), wsum (device) and q2 (host).  prm->sigma is ignored.  Here and in
 * kot_residual, kot_ssn_direction, kot_eg_step and kot_features, an R with a nonzero entry below its
 * diagonal is rejected with KOT_ERR_ARG (the products with R skip its zero triangle). */
kot_status kot_solve_core(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, double q2,
                          const double* wsum, const kot_params* prm, const double* gamma0, kot_result* res);

/* Symmetric eigendecomposition (Eq. 4.4): Z = P diag(w) P^T with w ascending.  Z, P (l x l) and w (l) are
 * device pointers; P's columns are the eigenvectors.  Z is not modified.  Returns KOT_ERR_NUMERIC if Z has a
 * non-finite entry (P, w then hold no result) and KOT_ERR_EIG if the
 * Jacobi sweeps do not reach the off-diagonal tolerance within prm->eig_max_sweeps (P, w still written). */
kot_status kot_eigh(kot_ctx* ctx, int l, const double* Z, double* P, double* w, const kot_params* prm);

/* kot_eigh for callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): no context, no hipMalloc/hipFree.  Its working storage is a static device
 * array of each GPU the library runs on (4.2 MiB, held until the process ends), so l is limited to
 * 1 <= l <= 512 (KOT_ERR_ARG beyond, with a message from kot_last_error(NULL)).  device: HIP device index
 * (made current for the call, the previous device restored); hip_stream: a hipStream_t on that device
 * (NULL = its default stream), synchronized before return.  Z, P (l x l) and w (l) are device pointers as in
 * kot_eigh; the cold-start Jacobi sweeps are full tournaments.  Every call on a GPU shares that GPU's array and
 * leaves the last call's contents in it: calls that overlap on one GPU (other threads or streams) race. */
kot_status kot_eigh_noalloc(int device, void* hip_stream, int l, const double* Z, double* P, double* w,
                            const kot_params* prm);

/* Residual map Eq. (4.2) at w = (gamma, X): r1 = (Q gamma - z)/(2 lambda2) - Phi(X),
 * r2 = X - Pi(X - Phi*(gamma) - lambda1 I), with Phi(X)_i = R[:,i]^T X R[:,i], Phi*(gamma) = R diag(gamma) R^T.
 * Q, z, R, gamma, X, r1, r2 are device pointers; norms (host, 3 entries) receives |r1|_2, |r2|_F and
 * the number of positive eigenvalues of Z (as a double). */
kot_status kot_residual(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R,
                        const double* gamma, const double* X, const kot_params* prm,
                        double* r1, double* r2, double* norms);

/* One regularized SSN direction (Eq. 4.3) by Algorithm 1 at w = (gamma, X) with regularization mu:
 * writes dgamma (device, l) and dX (device, l x l).  info (host, 4 entries): CG iterations, CG residual
 * norm, |alpha|, |r|. */
kot_status kot_ssn_direction(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R,
                             const double* gamma, const double* X, double mu, const kot_params* prm,
                             double* dgamma, double* dX, double* info);

/* The Schur operator of Algorithm 1 at w = (gamma, X) with regularization mu (Lemma 4.3):
 * y = (Q/(2 lambda2) + mu I + Phi T Phi*) v, T from the spectral data of Z = X - Phi*(gamma) - lambda1 I
 * (Section 4.3), applied through the eigen-row chain with B = P^T R in the precision prm->precision
 * (FP64; FP32; BF16 or split BF16 on the matrix cores with FP32 accumulation).  v, y (l) and Q, z, R, gamma,
 * X as in kot_ssn_direction (device).  The product runs `reps` times on the same v (reps >= 1, for timing; y
 * is overwritten each time).  info (host, 4 entries): |alpha|, the chain's row count
 * min(|alpha|, l - |alpha|), 1 if the complement form ran, and the mean milliseconds per product. */
kot_status kot_schur_matvec(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R,
                            const double* gamma, const double* X, double mu, const kot_params* prm, int reps,
                            const double* v, double* y, double* info);

/* One extragradient step (Section 4.4) on the min-max form Eq. (4.1) with step eta: (gamma, X) ->
 * (gamma_out, X_out), projection onto R^l x S^l_+.  All arrays device pointers. */
kot_status kot_eg_step(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R,
                       const double* gamma, const double* X, double eta, const kot_params* prm,
                       double* gamma_out, double* X_out);

/* Upper Cholesky factor R (device, l x l) of the symmetric positive definite A (device, l x l) + eps I:
 * R^T R = A + eps I; strictly lower triangle written as 0.  Rit (device, l x l) may be NULL; else it
 * receives R^-T, lower triangular with zeros above, formed by the same launches one block row behind the
 * factor (the lifted start of Section 5 needs it).  Returns KOT_ERR_FACTOR on a non-positive pivot (Rit
 * then undefined). */
kot_status kot_cholesky(kot_ctx* ctx, int l, const double* A, double eps, double* R, double* Rit);

/* General FP64 product on the device (MFMA): C = alpha op(A) diag(s) op(B) + beta C, op = transpose if
 * trans* != 0; s (device, length k) may be NULL.  C is m x n with leading dimension ldc.  The solver's product
 * modes, exposed for testing: tri declares known zero triangles (bit 1: op(A) upper triangular, 2: op(A) lower,
 * 4: op(B) upper, 8: op(B) lower; the skipped entries must be zero), sym declares a symmetric result (m == n,
 * and C symmetric when beta != 0): only the lower tiles are computed and mirrored.  KOT_ERR_ARG otherwise. */
kot_status kot_gemm(kot_ctx* ctx, int transa, int transb, int m, int n, int k, double alpha,
                    const double* A, int lda, const double* s, const double* B, int ldb, double beta,
                    double* C, int ldc, int tri, int sym);

/* ---- Learned warm start (not in the paper: a network predicting the start dual) ----------------------------
 * Network: f(x) = W3^T relu(W2^T relu(W1^T x + b1) + b2) + b3 applied to each row x of a feature matrix.
 * Parameters are one flat FP32 device vector theta of kot_mlp_params(F, H) entries laid out W1 (F x H,
 * row-major), b1 (H), W2 (H x H), b2 (H), W3 (H), b3 (1).  The prediction for filling point i is
 * gamma0_i = lambda1 * f(x_i).  Features (F = 12 per filling point, FP32, row-major l x 12), bounded and free of
 * the problem's scale, with f0 = z_i/(lambda1 Q_ii) and K = R^T R: max(f0,-2), max(f0,-1), (Q 1)_i/Q_ii - 1,
 * (K 1)_i/K_ii - 1, ((K o K) 1)_i/K_ii^2 - 1, Q_ii - 2, K_ii - 1, min(wsum_i/|z_i|, 10), the fraction of points
 * with f0 < -1, the mean of max(f0,-1), 0, 1.
 * Callers: training and inference of the warm start.  All matrices FP64 device, features/theta FP32 device. */
int kot_mlp_params(int F, int H);
kot_status kot_features(kot_ctx* ctx, int l, const double* Q, const double* z, const double* R, const double* wsum,
                        double q2, const kot_params* prm, float* X);
/* out (device, n) = f(X) for X (device, n x F). */
kot_status kot_mlp_forward(kot_ctx* ctx, int n, int F, int H, const float* X, const float* theta, float* out);
/* loss (host) = mean((f(X) - y)^2); grad (device, same layout as theta) = its gradient. */
kot_status kot_mlp_loss_grad(kot_ctx* ctx, int n, int F, int H, const float* X, const float* y, const float* theta,
                             float* grad, double* loss);
/* One Adam step on theta with moments m, v (device, P entries each); t = step count after this update (>= 1). */
kot_status kot_mlp_adam(kot_ctx* ctx, int P, float* theta, const float* grad, float* m, float* v, int t, float lr,
                        float beta1, float beta2, float eps);
/* gamma0 (device, l) predicted for the problem: runs the setup, the features and the network. */
kot_status kot_warmstart(kot_ctx* ctx, const kot_problem* prob, const kot_params* prm, int F, int H,
                         const float* theta, double* gamma0);

/* Kantorovich potentials and transport map of a solved problem (Section 3): with the dual gamma (device, l)
 * returned by kot_solve for the same problem and parameters, the maximizers of Eq. (3.2) are
 *   u(x) = (w_mu(x) - sum_i gamma_i k(xf_i, x)) / (2 lambda2),  v(y) = (w_nu(y) - sum_i gamma_i k(yf_i, y)) / (2 lambda2),
 * w_mu(x) = (1/n_src) sum_j k(xs_j, x), and for the cost |x - y|^2/2 the map T(x) = x - grad u(x).
 * xq, yq: m query points (device, m x d, row-major; either may be NULL); u, v (device, m) receive u(xq), v(yq);
 * Tx (device, m x d, may be NULL; needs xq) receives T(xq).  d <= 64.  Deterministic (fixed-order sums).
 * The context keeps a workspace of about 1024 x 17 doubles per 256 queries (grown on demand). */
kot_status kot_potentials(kot_ctx* ctx, const kot_problem* prob, const kot_params* prm, const double* gamma, int m,
                          const double* xq, const double* yq, double* u, double* v, double* Tx);

/* Launch profiler for measurement.  enable = 1 clears and starts recording HIP events around every launch
 * of the instrumented kernel classes on the context's stream; enable = 0 stops, waits for the stream, and
 * writes 4 values per class into out (host, 4 * nclass doubles; may be NULL): launches, total milliseconds
 * between the events, algorithmic flops and algorithmic bytes.  Classes: 0 = FP64 GEMM (2mnk flops),
 * 1 = one Jacobi sweep (all rounds of pair solves + tile updates, replayed as one captured HIP graph; flops of
 * the 16x16 tile products), 2 = FP64 matrix-vector product (2mk flops, bytes of the matrix and vectors),
 * 3 = FP32 chain GEMM, 4 = BF16 chain GEMM (2mnk flops each), 5 = potential evaluation (kot_potentials;
 * (6d + 3) flops per query-source pair, counting the exponential as one). */
kot_status kot_profile(kot_ctx* ctx, int enable, double* out, int nclass);

#ifdef __cplusplus
}
#endif
#endif /* KOTSSN_H */
