// Elementwise kernels, deterministic reductions and the Hadamard weight Psi of Section 4.3.
#include "kot_internal.h"

namespace kot {
namespace {

// y = x, two doubles per thread (a kernel: cheaper to enqueue than a runtime copy)
__global__ void copy_kernel(long long n, const double* __restrict__ x, double* __restrict__ y) {
  const long long i = 2 * ((long long)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 1 < n) {
    const double2 v = *reinterpret_cast<const double2*>(x + i);
    *reinterpret_cast<double2*>(y + i) = v;
  } else if (i < n) {
    y[i] = x[i];
  }
}

__global__ void fill_kernel(long long n, double v, double* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
__global__ void fill2d_kernel(int rows, int cols, double v, double* __restrict__ C, int ldc) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)rows * cols) return;
  C[(u / cols) * ldc + (u % cols)] = v;
}
__global__ void axpby_kernel(long long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
__global__ void lincomb_kernel(long long n, double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                               double* __restrict__ z) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = a * x[i] + b * y[i];
}
__global__ void add_diag_kernel(int l, double a, double* __restrict__ X) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < l) X[(long long)i * l + i] += a;
}
__global__ void symmetrize_kernel(int l, double* __restrict__ Z) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  if (j <= i) return;
  const double v = 0.5 * (Z[u] + Z[(long long)j * l + i]);
  Z[u] = v;
  Z[(long long)j * l + i] = v;
}
// Partial dot products of one or two vector pairs over a grid-stride slice, four loads in flight per pass;
// part[2 b] (and part[2 b + 1]) per block, fixed order.
__global__ __launch_bounds__(256) void dot2_part_kernel(long long n, const double* __restrict__ x1, const double* __restrict__ y1,
                                                        const double* __restrict__ x2, const double* __restrict__ y2,
                                                        double* __restrict__ part) {
  __shared__ double red[2][256];
  double a = 0.0, b = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i0 = (long long)blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    double u[4], v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long i = i0 + q * stride;
      u[q] = (i < n) ? x1[i] * y1[i] : 0.0;
      v[q] = (x2 && i < n) ? x2[i] * y2[i] : 0.0;
    }
    a += (u[0] + u[1]) + (u[2] + u[3]);
    b += (v[0] + v[1]) + (v[2] + v[3]);
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { red[0][threadIdx.x] += red[0][threadIdx.x + h]; red[1][threadIdx.x] += red[1][threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = red[0][0]; part[2 * blockIdx.x + 1] = red[1][0]; }
}
__global__ __launch_bounds__(256) void dot2_final_kernel(int nb, const double* __restrict__ part, double* __restrict__ o1,
                                                         double* __restrict__ o2) {
  __shared__ double red[2][256];
  red[0][threadIdx.x] = (threadIdx.x < nb) ? part[2 * threadIdx.x] : 0.0;
  red[1][threadIdx.x] = (threadIdx.x < nb) ? part[2 * threadIdx.x + 1] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { red[0][threadIdx.x] += red[0][threadIdx.x + h]; red[1][threadIdx.x] += red[1][threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    o1[0] = red[0][0];
    if (o2) o2[0] = red[1][0];
  }
}
// out = X - Y with the block partials of |out|^2 (the layout of dot2_part's first sum), in one pass.
__global__ __launch_bounds__(256) void sub_sq_part_kernel(long long n, const double* __restrict__ X,
                                                          const double* __restrict__ Y, double* __restrict__ out,
                                                          double* __restrict__ part) {
  __shared__ double red[256];
  double a = 0.0;
  const long long stride = (long long)gridDim.x * 256;
  for (long long i0 = (long long)blockIdx.x * 256 + threadIdx.x; i0 < n; i0 += 4 * stride) {
    double u[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const long long i = i0 + q * stride;
      u[q] = 0.0;
      if (i < n) {
        const double d = X[i] - Y[i];
        out[i] = d;
        u[q] = d * d;
      }
    }
    a += (u[0] + u[1]) + (u[2] + u[3]);
  }
  red[threadIdx.x] = a;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) { part[2 * blockIdx.x] = red[0]; part[2 * blockIdx.x + 1] = 0.0; }
}

// o1 = |r1|^2 (length l) and o2 = the sum of the nb first-sum partials, fixed order throughout.
__global__ __launch_bounds__(256) void resid_final_kernel(int nb, const double* __restrict__ part, int l,
                                                          const double* __restrict__ r1, double* __restrict__ o1,
                                                          double* __restrict__ o2) {
  __shared__ double red[2][256];
  double q[4] = {0.0, 0.0, 0.0, 0.0};
  int i = threadIdx.x;
  for (; i + 768 < l; i += 1024)
#pragma unroll
    for (int u = 0; u < 4; ++u) q[u] += r1[i + 256 * u] * r1[i + 256 * u];
  for (; i < l; i += 256) q[0] += r1[i] * r1[i];
  red[0][threadIdx.x] = (q[0] + q[1]) + (q[2] + q[3]);
  red[1][threadIdx.x] = (threadIdx.x < nb) ? part[2 * threadIdx.x] : 0.0;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) { red[0][threadIdx.x] += red[0][threadIdx.x + h]; red[1][threadIdx.x] += red[1][threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    o1[0] = red[0][0];
    o2[0] = red[1][0];
  }
}

// Short vectors (n <= kSmallDot): one workgroup, eight loads in flight per thread, fixed order.
constexpr int kSmallDot = 8192;
__global__ __launch_bounds__(1024) void dot2_small_kernel(int n, const double* __restrict__ x1, const double* __restrict__ y1,
                                                          const double* __restrict__ x2, const double* __restrict__ y2,
                                                          double* __restrict__ o1, double* __restrict__ o2) {
  __shared__ double red[2][1024];
  double u[8], v[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = threadIdx.x + 1024 * q;
    u[q] = (i < n) ? x1[i] * y1[i] : 0.0;
    v[q] = (x2 && i < n) ? x2[i] * y2[i] : 0.0;
  }
  red[0][threadIdx.x] = ((u[0] + u[1]) + (u[2] + u[3])) + ((u[4] + u[5]) + (u[6] + u[7]));
  red[1][threadIdx.x] = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (threadIdx.x < h) { red[0][threadIdx.x] += red[0][threadIdx.x + h]; red[1][threadIdx.x] += red[1][threadIdx.x + h]; }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    o1[0] = red[0][0];
    if (o2) o2[0] = red[1][0];
  }
}
// Z = sym(X - a T) + c I with sym(M) = (M + M^T)/2: one workgroup per 32x32 tile pair (I, J), I <= J, both
// tiles staged in LDS so the transposed reads stay coalesced; Z is exactly symmetric.
__global__ __launch_bounds__(256) void form_z_kernel(int l, const double* __restrict__ X, double a,
                                                     const double* __restrict__ T, double c, double* __restrict__ Z) {
  const int I = blockIdx.y, J = blockIdx.x;
  if (J < I) return;
  __shared__ double mij[32][33], mji[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double u[4], v[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = I * 32 + r, j = J * 32 + tx;
    u[q] = (i < l && j < l) ? X[(long long)i * l + j] - a * T[(long long)i * l + j] : 0.0;
    const int i2 = J * 32 + r, j2 = I * 32 + tx;
    v[q] = (i2 < l && j2 < l) ? X[(long long)i2 * l + j2] - a * T[(long long)i2 * l + j2] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    mij[ty + 8 * q][tx] = u[q];
    mji[ty + 8 * q][tx] = v[q];
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = ty + 8 * q;
    const int i = I * 32 + r, j = J * 32 + tx;
    if (i < l && j < l) {
      double z = 0.5 * (mij[r][tx] + mji[tx][r]);
      if (i == j) z += c;
      Z[(long long)i * l + j] = z;
    }
    const int i2 = J * 32 + r, j2 = I * 32 + tx;
    if (I != J && i2 < l && j2 < l) Z[(long long)i2 * l + j2] = 0.5 * (mji[r][tx] + mij[tx][r]);
  }
}

// CG update with the step length on the device: alpha = rr / pAp (0 if pAp <= 0, which the host then sees);
// x += alpha p, r -= alpha Ap.
__global__ void cg_step_kernel(int n, double rr, const double* __restrict__ pAp, const double* __restrict__ p,
                               const double* __restrict__ Ap, double* __restrict__ x, double* __restrict__ r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double d = *pAp;
  const double alpha = (d > 0.0) ? rr / d : 0.0;
  x[i] = alpha * p[i] + x[i];
  r[i] = -alpha * Ap[i] + r[i];
}
// ---- conjugate gradients with the scalars on the device ------------------------------------------------------
// st: [CG_RR] r.r, [CG_XX] x.x, [CG_DONE] 0 running / 1 stopped, [CG_IT] iterations done, [CG_RZ] r.D^-1 r
// with a diagonal preconditioner D (dinv = D^-1 non-null; preconditioned CG: z = D^-1 r, alpha = r.z / p.Ap,
// beta = r'.z' / r.z, p = z + beta p).  The stopping test is Eq. (4.5)'s on the unpreconditioned residual:
// |r| <= thr with thr = tau min(1, kr |x|) (kr = kappa |R(w)|), or a fixed thr when fixed > 0; an iteration
// count reaching cap, or a non-positive p.Ap, stops as well.  Iterations queued after the stop leave every
// vector unchanged, so the host may queue several before it looks.
constexpr int CG_RR = 0, CG_XX = 1, CG_DONE = 2, CG_IT = 3, CG_RZ = 4;

// Sums of three values over a 1024-thread workgroup, the same on every thread (shuffles inside each wavefront,
// then the sixteen wavefront partials in a fixed order).
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double (*sh)[16]) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c += __shfl_xor(c, o);
  }
  const int w = threadIdx.x >> 6;
  __syncthreads();  // earlier readers of sh are done
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
    sh[2][w] = c;
  }
  __syncthreads();
  a = b = c = 0.0;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    a += sh[0][k];
    b += sh[1][k];
    c += sh[2][k];
  }
}

__device__ __forceinline__ bool cg_stop(double rr, double xx, double tau, double kr, double fixed) {
  const double thr = fixed > 0.0 ? fixed : tau * fmin(1.0, kr * sqrt(xx));
  return sqrt(rr) <= thr;
}

// x = 0, r = b, p = D^-1 b (b without a preconditioner), r.r, r.z, and the stopping test at the start.
__global__ __launch_bounds__(1024) void cg_init_kernel(int n, const double* __restrict__ b, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ p,
                                                       double* __restrict__ st, double tau, double kr, double fixed,
                                                       int cap, const double* __restrict__ dinv) {
  __shared__ double sh[3][16];
  double rr = 0.0, rz = 0.0, z2 = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = threadIdx.x + 1024 * q;
    if (i < n) {
      const double v = b[i];
      const double z = dinv ? dinv[i] * v : v;
      x[i] = 0.0;
      r[i] = v;
      p[i] = z;
      rr += v * v;
      rz += v * z;
    }
  }
  block_sum3(rr, rz, z2, sh);
  if (threadIdx.x == 0) {
    st[CG_RR] = rr;
    st[CG_RZ] = rz;
    st[CG_XX] = 0.0;
    st[CG_IT] = 0.0;
    st[CG_DONE] = (cap <= 0 || cg_stop(rr, 0.0, tau, kr, fixed)) ? 1.0 : 0.0;
  }
}

// The vector part of one iteration, Ap (+ addmu p) given:  alpha = r.r / p.Ap;  x += alpha p;  r -= alpha Ap;
// p = r + (r'.r' / r.r) p; then the stopping test on the new r and x.
__global__ __launch_bounds__(1024) void cg_tail_kernel(int n, double* __restrict__ st, double* __restrict__ p,
                                                       const double* __restrict__ Ap, double addmu,
                                                       double* __restrict__ x, double* __restrict__ r, double tau,
                                                       double kr, double fixed, int cap,
                                                       const double* __restrict__ dinv) {
  __shared__ double sh[3][16];
  if (st[CG_DONE] != 0.0) return;
  const double rr = st[CG_RR];
  const double rz = dinv ? st[CG_RZ] : rr;
  double pv[8], av[8];
  double pap = 0.0, z1 = 0.0, z2 = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = threadIdx.x + 1024 * q;
    pv[q] = (i < n) ? p[i] : 0.0;
    av[q] = (i < n) ? addmu * pv[q] + Ap[i] : 0.0;
    pap += pv[q] * av[q];
  }
  block_sum3(pap, z1, z2, sh);
  if (!(pap > 0.0)) {  // breakdown: stop with x and r as they are
    if (threadIdx.x == 0) st[CG_DONE] = 1.0;
    return;
  }
  const double alpha = rz / pap;
  double rv[8];
  double rs = 0.0, xs = 0.0, rzn = 0.0;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = threadIdx.x + 1024 * q;
    rv[q] = 0.0;
    if (i < n) {
      const double xn = alpha * pv[q] + x[i];
      const double rn = -alpha * av[q] + r[i];
      x[i] = xn;
      r[i] = rn;
      rv[q] = dinv ? dinv[i] * rn : rn;  // z = D^-1 r
      rs += rn * rn;
      xs += xn * xn;
      rzn += rn * rv[q];
    }
  }
  block_sum3(rs, xs, rzn, sh);
  const double beta = dinv ? rzn / rz : rs / rr;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int i = threadIdx.x + 1024 * q;
    if (i < n) p[i] = beta * pv[q] + rv[q];
  }
  if (threadIdx.x == 0) {
    const double it = st[CG_IT] + 1.0;
    st[CG_IT] = it;
    st[CG_RR] = rs;
    st[CG_XX] = xs;
    st[CG_RZ] = rzn;
    if (it >= (double)cap || cg_stop(rs, xs, tau, kr, fixed)) st[CG_DONE] = 1.0;
  }
}

// ---- symmetric QMR (Freund and Nachtigal's simplified QMR) with the scalars on the device ------------------
// st as for CG ([CG_RR] holds s.s of the true residual s = b - A x, [CG_RZ] rho = r.D^-1 r) plus [SQ_TAU] tau and
// [SQ_THETA] theta.  Vectors: x, r (the Lanczos / BCG residual), q (direction, the operand of the product),
// d (the last update of x), e = A d, s = b - A x.  Same stopping test as CG, on s.
constexpr int SQ_TAU = 5, SQ_THETA = 6;

__global__ __launch_bounds__(1024) void sqmr_init_kernel(int n, const double* __restrict__ b, double* __restrict__ x,
                                                         double* __restrict__ r, double* __restrict__ q,
                                                         double* __restrict__ d, double* __restrict__ e,
                                                         double* __restrict__ s, double* __restrict__ st, double tau,
                                                         double kr, double fixed, int cap,
                                                         const double* __restrict__ dinv) {
  __shared__ double sh[3][16];
  double bb = 0.0, rho = 0.0, z2 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = threadIdx.x + 1024 * k;
    if (i < n) {
      const double v = b[i];
      const double u = dinv ? dinv[i] * v : v;
      x[i] = 0.0;
      d[i] = 0.0;
      e[i] = 0.0;
      r[i] = v;
      s[i] = v;
      q[i] = u;
      bb += v * v;
      rho += v * u;
    }
  }
  block_sum3(bb, rho, z2, sh);
  if (threadIdx.x == 0) {
    st[CG_RR] = bb;
    st[CG_XX] = 0.0;
    st[CG_IT] = 0.0;
    st[CG_RZ] = rho;
    st[SQ_TAU] = sqrt(rho);
    st[SQ_THETA] = 0.0;
    st[CG_DONE] = (cap <= 0 || cg_stop(bb, 0.0, tau, kr, fixed)) ? 1.0 : 0.0;
  }
}

// One iteration given t = A q.  A non-positive q.t or rho stops (the operator is SPD; neither happens in exact
// arithmetic).
__global__ __launch_bounds__(1024) void sqmr_tail_kernel(int n, double* __restrict__ st, double* __restrict__ q,
                                                         const double* __restrict__ t, double* __restrict__ x,
                                                         double* __restrict__ r, double* __restrict__ d,
                                                         double* __restrict__ e, double* __restrict__ s, double tau,
                                                         double kr, double fixed, int cap,
                                                         const double* __restrict__ dinv) {
  __shared__ double sh[3][16];
  if (st[CG_DONE] != 0.0) return;
  const double rho = st[CG_RZ];
  double qv[8], tv[8];
  double sigma = 0.0, z1 = 0.0, z2 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = threadIdx.x + 1024 * k;
    qv[k] = (i < n) ? q[i] : 0.0;
    tv[k] = (i < n) ? t[i] : 0.0;
    sigma += qv[k] * tv[k];
  }
  block_sum3(sigma, z1, z2, sh);
  if (!(sigma > 0.0) || !(rho > 0.0)) {
    if (threadIdx.x == 0) st[CG_DONE] = 1.0;
    return;
  }
  const double alpha = rho / sigma;
  double rv[8], uv[8];
  double rho_n = 0.0, z3 = 0.0, z4 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = threadIdx.x + 1024 * k;
    rv[k] = 0.0;
    uv[k] = 0.0;
    if (i < n) {
      rv[k] = -alpha * tv[k] + r[i];
      uv[k] = dinv ? dinv[i] * rv[k] : rv[k];
      r[i] = rv[k];
      rho_n += rv[k] * uv[k];
    }
  }
  block_sum3(rho_n, z3, z4, sh);
  const double theta_o = st[SQ_THETA];
  const double theta = sqrt(rho_n) / st[SQ_TAU];
  const double c2 = 1.0 / (1.0 + theta * theta);
  const double taun = st[SQ_TAU] * theta * sqrt(c2);
  const double fd = c2 * theta_o * theta_o, fq = c2 * alpha, beta = rho_n / rho;
  double ss = 0.0, xx = 0.0, z5 = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int i = threadIdx.x + 1024 * k;
    if (i < n) {
      const double dn = fd * d[i] + fq * qv[k];
      const double en = fd * e[i] + fq * tv[k];
      const double xn = x[i] + dn;
      const double sn = s[i] - en;
      d[i] = dn;
      e[i] = en;
      x[i] = xn;
      s[i] = sn;
      q[i] = uv[k] + beta * qv[k];
      ss += sn * sn;
      xx += xn * xn;
    }
  }
  block_sum3(ss, xx, z5, sh);
  if (threadIdx.x == 0) {
    const double it = st[CG_IT] + 1.0;
    st[CG_IT] = it;
    st[CG_RR] = ss;
    st[CG_XX] = xx;
    st[CG_RZ] = rho_n;
    st[SQ_TAU] = taun;
    st[SQ_THETA] = theta;
    if (it >= (double)cap || cg_stop(ss, xx, tau, kr, fixed)) st[CG_DONE] = 1.0;
  }
}

// d_i = cq Q_ii + mu + ckk KK_ii (KK may be null): the Schur operator's diagonal outside its eigen-chain term.
__global__ void schur_diag_base_kernel(int l, const double* __restrict__ Q, double cq, double mu,
                                       const double* __restrict__ KK, double ckk, double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const long long ii = (long long)i * l + i;
  d[i] = cq * Q[ii] + mu + (KK ? ckk * KK[ii] : 0.0);
}

// out_i = 1 / d_i
__global__ void recip_kernel(int n, const double* __restrict__ d, double* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = 1.0 / d[i];
}

__global__ __launch_bounds__(256) void rowsum_abs_kernel(int l, const double* __restrict__ A, int sq, double* __restrict__ rows) {
  __shared__ double red[256];
  const int i = blockIdx.x;
  double acc = 0.0;
  for (int j = threadIdx.x; j < l; j += 256) {
    const double v = A[(long long)i * l + j];
    acc += sq ? v * v : fabs(v);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) rows[i] = red[0];
}
__global__ __launch_bounds__(256) void max_kernel(int n, const double* __restrict__ v, double* __restrict__ out) {
  __shared__ double red[256];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) m = fmax(m, v[i]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
__global__ void fill_int_kernel(int* __restrict__ out) { out[0] = 0; }

__global__ __launch_bounds__(256) void count_pos_kernel(int l, const double* __restrict__ w, int* __restrict__ out) {
  __shared__ int red[256];
  int c = 0;
  for (int i = threadIdx.x; i < l; i += 256) c += (w[i] > 0.0) ? 1 : 0;
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

// out[0] += number of nonzero entries strictly below the diagonal (one 256-row slab per workgroup column)
__global__ __launch_bounds__(256) void count_lower_kernel(int l, const double* __restrict__ R, int* __restrict__ out) {
  __shared__ int red[256];
  int c = 0;
  for (long long u = (long long)blockIdx.x * 256 + threadIdx.x; u < (long long)l * l; u += (long long)gridDim.x * 256) {
    const int i = (int)(u / l), j = (int)(u - (long long)i * l);
    if (j < i && R[u] != 0.0) ++c;
  }
  red[threadIdx.x] = c;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0 && red[0]) atomicAdd(out, red[0]);
}

// Psi weights (Section 4.3), eigenvalues w ascending so alpha = [l-a, l).
//   non-complement, row r in alpha:  j in alpha -> diag_scale/mu ;  j not in alpha -> off_scale * xi(r, j)
//   complement, row r not in alpha:  j not in alpha -> diag_scale/mu ; j in alpha -> off_scale * (1/mu - xi(j, r))
// with eta(i, j) = w_i/(w_i - w_j) (i in alpha, j not), 1 - eta = |w_j|/(w_i + |w_j|), xi = eta/(mu + 1 - eta),
// and 1/mu - xi = (1 - eta)(1 + mu) / (mu (mu + 1 - eta)).
__global__ void psi_kernel(int l, int a, int r0, int m, double mu, const double* __restrict__ w, double* __restrict__ C, int ldc,
                           int complement, double diag_scale, double off_scale) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)m * l) return;
  const int rr = (int)(u / l), j = (int)(u % l);
  const int r = r0 + rr;
  const int split = l - a;  // first alpha index
  const bool r_in = r >= split, j_in = j >= split;
  double wt;
  if (r_in == j_in) {
    wt = diag_scale / mu;
  } else {
    const int ia = r_in ? r : j;   // alpha member
    const int ib = r_in ? j : r;   // alpha-bar member
    const double sa = w[ia], sb = -w[ib];       // sa > 0, sb >= 0
    const double one_m_eta = sb / (sa + sb);
    const double eta = sa / (sa + sb);
    if (!complement) wt = off_scale * (eta / (mu + one_m_eta));
    else wt = off_scale * (one_m_eta * (1.0 + mu) / (mu * (mu + one_m_eta)));
  }
  C[(long long)rr * ldc + j] *= wt;
}

__global__ void sub_kernel(long long n, const double* __restrict__ X, const double* __restrict__ Y, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = X[i] - Y[i];
}
__global__ void transpose_kernel(int l, const double* __restrict__ A, double* __restrict__ At) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads = 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int i = by + k, j = bx + tx;
    if (i < l && j < l) tile[k][tx] = A[(long long)i * l + j];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int i = bx + k, j = by + tx;
    if (i < l && j < l) At[(long long)i * l + j] = tile[tx][k];
  }
}
__global__ void hsq_kernel(long long n, const double* __restrict__ A, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = A[i] * A[i];
}
__global__ void sym_plus_kernel(int l, const double* __restrict__ G, double a, const double* __restrict__ S, double b,
                                double* __restrict__ out) {
  __shared__ double tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  // tile holds G^T block: rows of the output block (by..), cols (bx..) need G[j][i]
  for (int k = ty; k < 32; k += 8) {
    const int i = bx + k, j = by + tx;  // read G[i][j] with i in col-range, j in row-range
    if (i < l && j < l) tile[tx][k] = G[(long long)i * l + j];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int i = by + k, j = bx + tx;
    if (i < l && j < l) {
      const long long u = (long long)i * l + j;
      const double g = G[u] + tile[k][tx];
      out[u] = (b == 0.0 || S == nullptr) ? a * g : a * g + b * S[u];
    }
  }
}
__global__ void scale_cols_kernel(int rows, int cols, const double* __restrict__ A, int lda, const double* __restrict__ s,
                                  double* __restrict__ out, int ldo) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)rows * cols) return;
  const int i = (int)(u / cols), j = (int)(u % cols);
  out[(long long)i * ldo + j] = A[(long long)i * lda + j] * s[j];
}

// ---- diagonal kernel factor (Remark 4.5: sparsity of K) ------------------------------------------------------
// out[0] = max_{i != j} |A_ij|, out[1] = max_i |A_ii|; out must hold zeros on entry (atomic max on the bit
// patterns of non-negative doubles, which order like the values).  One row per workgroup.
__global__ __launch_bounds__(256) void offdiag_absmax_kernel(int l, const double* __restrict__ A, double* out) {
  const int i = blockIdx.x;
  double m = 0.0, dm = 0.0;
  for (int j = threadIdx.x; j < l; j += 256) {
    const double v = fabs(A[(long long)i * l + j]);
    if (j == i) dm = v;
    else m = fmax(m, v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    m = fmax(m, __shfl_xor(m, o));
    dm = fmax(dm, __shfl_xor(dm, o));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(reinterpret_cast<unsigned long long*>(out), (unsigned long long)__double_as_longlong(m));
    atomicMax(reinterpret_cast<unsigned long long*>(out + 1), (unsigned long long)__double_as_longlong(dm));
  }
}

// R = diag(sqrt(K_ii)) (dense l x l, zeros off the diagonal), rd_i = R_ii, Linv = R^-T when non-null; info = 0,
// then (diag_check_kernel) an index (1-based) with K_ii <= 0, if any.
__global__ void diag_factor_kernel(int l, const double* __restrict__ K, double* __restrict__ R, double* __restrict__ rd,
                                   double* __restrict__ Linv, int* __restrict__ info) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u == 0) *info = 0;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  double r = 0.0, ri = 0.0;
  if (i == j) {
    const double k = K[u];
    r = sqrt(k);
    ri = 1.0 / r;
    rd[i] = r;
  }
  R[u] = r;
  if (Linv) Linv[u] = ri;
}
__global__ void diag_check_kernel(int l, const double* __restrict__ K, int* __restrict__ info) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < l && !(K[(long long)i * l + i] > 0.0)) atomicCAS(info, 0, i + 1);
}

// out = diag(rd_i^2 g_i) (power 2) or diag(g_i / rd_i^2) (power -2), dense l x l.
__global__ void diag_gram_kernel(int l, const double* __restrict__ rd, int power, const double* __restrict__ g,
                                 double* __restrict__ out) {
  const long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= (long long)l * l) return;
  const int i = (int)(u / l), j = (int)(u % l);
  double v = 0.0;
  if (i == j) v = power > 0 ? rd[i] * rd[i] * g[i] : g[i] / (rd[i] * rd[i]);
  out[u] = v;
}

// y_i = alpha rd_i^2 X_ii + beta y_i (beta = 0: y is not read).
__global__ void phi_diag_kernel(int l, const double* __restrict__ rd, const double* __restrict__ X, double alpha,
                                double beta, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= l) return;
  const double v = alpha * rd[i] * rd[i] * X[(long long)i * l + i];
  y[i] = beta != 0.0 ? v + beta * y[i] : v;
}

// B = P^T diag(rd): B_ij = P_ji rd_j, through 32 x 32 LDS tiles (coalesced reads and writes).
__global__ __launch_bounds__(256) void transpose_scale_kernel(int l, const double* __restrict__ P,
                                                              const double* __restrict__ rd, double* __restrict__ B) {
  __shared__ double T[32][33];
  const int bi = blockIdx.y * 32, bj = blockIdx.x * 32;  // the B tile (rows bi.., columns bj..)
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {  // P rows bj + r, columns bi + tx
    const int pr = bj + r, pc = bi + tx;
    T[r][tx] = (pr < l && pc < l) ? P[(long long)pr * l + pc] * rd[pr] : 0.0;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int br = bi + r, bc = bj + tx;
    if (br < l && bc < l) B[(long long)br * l + bc] = T[tx][r];
  }
}

inline int nblk(long long n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace

hipError_t vec_fill(int n, double v, double* x, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(nblk(n)), dim3(256), 0, st, (long long)n, v, x);
  return hipGetLastError();
}
hipError_t mat_fill(int rows, int cols, double v, double* C, int ldc, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill2d_kernel, dim3(nblk((long long)rows * cols)), dim3(256), 0, st, rows, cols, v, C, ldc);
  return hipGetLastError();
}
hipError_t vec_copy(int n, const double* x, double* y, hipStream_t st) {
  if (n <= 0 || x == y) return hipSuccess;
  // double2 accesses need 16-byte alignment of both; otherwise the runtime copy
  if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) & 15)
    return hipMemcpyAsync(y, x, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, st);
  const long long pairs = ((long long)n + 1) / 2;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)((pairs + 255) / 256)), dim3(256), 0, st, (long long)n, x, y);
  return hipGetLastError();
}
hipError_t vec_axpby(int n, double a, const double* x, double b, double* y, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(nblk(n)), dim3(256), 0, st, (long long)n, a, x, b, y);
  return hipGetLastError();
}
hipError_t vec_lincomb(int n, double a, const double* x, double b, const double* y, double* z, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n)), dim3(256), 0, st, (long long)n, a, x, b, y, z);
  return hipGetLastError();
}
hipError_t offdiag_absmax(int l, const double* A, double* out, hipStream_t st) {
  hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(256), 0, st, 2LL, 0.0, out);
  hipLaunchKernelGGL(offdiag_absmax_kernel, dim3(l), dim3(256), 0, st, l, A, out);
  return hipGetLastError();
}
hipError_t diag_factor(int l, const double* K, double* R, double* rd, double* Linv, int* info, hipStream_t st) {
  hipLaunchKernelGGL(diag_factor_kernel, dim3(nblk((long long)l * l)), dim3(256), 0, st, l, K, R, rd, Linv, info);
  hipLaunchKernelGGL(diag_check_kernel, dim3(nblk(l)), dim3(256), 0, st, l, K, info);
  return hipGetLastError();
}
hipError_t diag_gram(int l, const double* rd, int power, const double* g, double* out, hipStream_t st) {
  hipLaunchKernelGGL(diag_gram_kernel, dim3(nblk((long long)l * l)), dim3(256), 0, st, l, rd, power, g, out);
  return hipGetLastError();
}
hipError_t phi_diag(int l, const double* rd, const double* X, double alpha, double beta, double* y, hipStream_t st) {
  hipLaunchKernelGGL(phi_diag_kernel, dim3(nblk(l)), dim3(256), 0, st, l, rd, X, alpha, beta, y);
  return hipGetLastError();
}
hipError_t transpose_scale(int l, const double* P, const double* rd, double* B, hipStream_t st) {
  const int t = (l + 31) / 32;
  hipLaunchKernelGGL(transpose_scale_kernel, dim3(t, t), dim3(256), 0, st, l, P, rd, B);
  return hipGetLastError();
}
hipError_t add_diag(int l, double a, double* X, hipStream_t st) {
  hipLaunchKernelGGL(add_diag_kernel, dim3(nblk(l)), dim3(256), 0, st, l, a, X);
  return hipGetLastError();
}
hipError_t symmetrize(int l, double* Z, hipStream_t st) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nblk((long long)l * l)), dim3(256), 0, st, l, Z);
  return hipGetLastError();
}
hipError_t dot2(long long n, const double* x1, const double* y1, double* o1, const double* x2, const double* y2,
               double* o2, double* part, hipStream_t st) {
  if (n <= kSmallDot) {
    hipLaunchKernelGGL(dot2_small_kernel, dim3(1), dim3(1024), 0, st, (int)n, x1, y1, x2, y2, o1, o2);
    return hipGetLastError();
  }
  long long nb = (n + 4 * 256 - 1) / (4 * 256);
  if (nb > kRedBlocks) nb = kRedBlocks;
  hipLaunchKernelGGL(dot2_part_kernel, dim3((unsigned)nb), dim3(256), 0, st, n, x1, y1, x2, y2, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(dot2_final_kernel, dim3(1), dim3(256), 0, st, (int)nb, part, o1, o2);
  return hipGetLastError();
}
int mat_sub_sq(long long n, const double* X, const double* Y, double* out, double* part, hipStream_t st) {
  long long nb = (n + 4 * 256 - 1) / (4 * 256);
  if (nb > kRedBlocks) nb = kRedBlocks;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(sub_sq_part_kernel, dim3((unsigned)nb), dim3(256), 0, st, n, X, Y, out, part);
  return hipGetLastError() == hipSuccess ? (int)nb : -1;
}
hipError_t resid_norms_final(int nb, const double* part, int l, const double* r1, double* o1, double* o2,
                             hipStream_t st) {
  hipLaunchKernelGGL(resid_final_kernel, dim3(1), dim3(256), 0, st, nb, part, l, r1, o1, o2);
  return hipGetLastError();
}
hipError_t dot(int n, const double* x, const double* y, double* out, double* part, hipStream_t st) {
  return dot2(n, x, y, out, nullptr, nullptr, nullptr, part, st);
}
hipError_t form_z(int l, const double* X, double a, const double* T, double c, double* Z, hipStream_t st) {
  const int nt = (l + 31) / 32;
  hipLaunchKernelGGL(form_z_kernel, dim3(nt, nt), dim3(256), 0, st, l, X, a, T, c, Z);
  return hipGetLastError();
}
hipError_t cg_init(int n, const double* b, double* x, double* r, double* p, double* st, double tau, double kr,
                   double fixed, int cap, hipStream_t st_, const double* dinv) {
  if (n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cg_init_kernel, dim3(1), dim3(1024), 0, st_, n, b, x, r, p, st, tau, kr, fixed, cap, dinv);
  return hipGetLastError();
}

hipError_t cg_tail(int n, double* st, double* p, const double* Ap, double addmu, double* x, double* r, double tau,
                   double kr, double fixed, int cap, hipStream_t st_, const double* dinv) {
  if (n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cg_tail_kernel, dim3(1), dim3(1024), 0, st_, n, st, p, Ap, addmu, x, r, tau, kr, fixed, cap,
                     dinv);
  return hipGetLastError();
}

hipError_t cg_step(int n, double rr, const double* pAp, const double* p, const double* Ap, double* x, double* r,
                   hipStream_t st) {
  hipLaunchKernelGGL(cg_step_kernel, dim3(nblk(n)), dim3(256), 0, st, n, rr, pAp, p, Ap, x, r);
  return hipGetLastError();
}
hipError_t sqmr_init(int n, const double* b, double* x, double* r, double* q, double* d, double* e, double* s,
                     double* st, double tau, double kr, double fixed, int cap, hipStream_t st_, const double* dinv) {
  if (n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sqmr_init_kernel, dim3(1), dim3(1024), 0, st_, n, b, x, r, q, d, e, s, st, tau, kr, fixed, cap,
                     dinv);
  return hipGetLastError();
}
hipError_t sqmr_tail(int n, double* st, double* q, const double* t, double* x, double* r, double* d, double* e,
                     double* s, double tau, double kr, double fixed, int cap, hipStream_t st_, const double* dinv) {
  if (n > 8192) return hipErrorInvalidValue;
  hipLaunchKernelGGL(sqmr_tail_kernel, dim3(1), dim3(1024), 0, st_, n, st, q, t, x, r, d, e, s, tau, kr, fixed, cap,
                     dinv);
  return hipGetLastError();
}
hipError_t schur_diag_base(int l, const double* Q, double cq, double mu, const double* KK, double ckk, double* d,
                           hipStream_t st) {
  hipLaunchKernelGGL(schur_diag_base_kernel, dim3((l + 255) / 256), dim3(256), 0, st, l, Q, cq, mu, KK, ckk, d);
  return hipGetLastError();
}
hipError_t vec_recip(int n, const double* d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(recip_kernel, dim3((n + 255) / 256), dim3(256), 0, st, n, d, out);
  return hipGetLastError();
}
hipError_t rowsum_abs_max(int l, const double* A, bool square_entries, double* out, double* part, hipStream_t st) {
  hipLaunchKernelGGL(rowsum_abs_kernel, dim3(l), dim3(256), 0, st, l, A, square_entries ? 1 : 0, part);
  KOT_HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(max_kernel, dim3(1), dim3(256), 0, st, l, part, out);
  return hipGetLastError();
}
hipError_t count_lower_nonzero(int l, const double* R, int* out_int, hipStream_t st) {
  hipLaunchKernelGGL(fill_int_kernel, dim3(1), dim3(1), 0, st, out_int);
  KOT_HIP_TRY(hipGetLastError());
  long long nb = ((long long)l * l + 255) / 256;
  if (nb > 1024) nb = 1024;
  hipLaunchKernelGGL(count_lower_kernel, dim3((unsigned)nb), dim3(256), 0, st, l, R, out_int);
  return hipGetLastError();
}
hipError_t count_positive(int l, const double* w, int* out_int, hipStream_t st) {
  hipLaunchKernelGGL(count_pos_kernel, dim3(1), dim3(256), 0, st, l, w, out_int);
  return hipGetLastError();
}
hipError_t psi_hadamard(int l, int a, int r0, int m, double mu, const double* w, double* C, int ldc, bool complement,
                        double diag_scale, double off_scale, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(psi_kernel, dim3(nblk((long long)m * l)), dim3(256), 0, st, l, a, r0, m, mu, w, C, ldc,
                     complement ? 1 : 0, diag_scale, off_scale);
  return hipGetLastError();
}
hipError_t mat_sub(int n, const double* X, const double* Y, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sub_kernel, dim3(nblk(n)), dim3(256), 0, st, (long long)n, X, Y, out);
  return hipGetLastError();
}
hipError_t transpose(int l, const double* A, double* At, hipStream_t st) {
  dim3 grid((l + 31) / 32, (l + 31) / 32);
  hipLaunchKernelGGL(transpose_kernel, grid, dim3(256), 0, st, l, A, At);
  return hipGetLastError();
}
hipError_t hadamard_square(int n, const double* A, double* out, hipStream_t st) {
  hipLaunchKernelGGL(hsq_kernel, dim3(nblk(n)), dim3(256), 0, st, (long long)n, A, out);
  return hipGetLastError();
}
hipError_t sym_plus(int l, const double* G, double a, const double* S, double b, double* out, hipStream_t st) {
  dim3 grid((l + 31) / 32, (l + 31) / 32);
  hipLaunchKernelGGL(sym_plus_kernel, grid, dim3(256), 0, st, l, G, a, S, b, out);
  return hipGetLastError();
}
hipError_t scale_cols(int rows, int cols, const double* A, int lda, const double* s, double* out, int ldo, hipStream_t st) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(nblk((long long)rows * cols)), dim3(256), 0, st, rows, cols, A, lda, s, out, ldo);
  return hipGetLastError();
}

}  // namespace kot
