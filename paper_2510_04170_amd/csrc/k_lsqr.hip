// LSQR (Paige and Saunders, ACM TOMS 8(1), 1982) on A = (D J) R^{-1}, the inner
// solver of Alg. 1 step 4 and Alg. 2 step 5, plus the small vector kernels of
// the Newton drivers.
//
// All scalars of the recurrence live in one LsqrState on the GPU; a one-block
// kernel reduces the norm partials in a fixed order and advances the state, so
// an iteration is a fixed chain of launches with no host round trip.  The
// unnormalised Golub-Kahan vectors u~ and v~ are stored with their norms beta
// and alpha, and the consumers scale on the fly:
//   p   = R^{-1} (v~ / alpha)
//   u~ <- D J p - (alpha / beta) u~,          beta  = ||u~||
//   q   = (D J)^T (u~ / beta)
//   v~ <- R^{-T} q - (beta / alpha) v~,       alpha = ||v~||
//   plane rotation, x += (phi/rho) w, w = v~/alpha - (theta/rho) w
// Once a stop rule fires the state's done flag turns every later launch of the
// chain into a no-op, so the host only polls it every few iterations.
#include <cmath>

#include "rfm_internal.h"

namespace rfm {

namespace {

constexpr int kB = 256;

enum Stage { kInitBeta = 0, kInitAlpha = 1, kBeta = 2, kAlpha = 3, kXnorm = 4 };

__device__ __forceinline__ double block_sum(const double* __restrict__ partials, int np, double* sh) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += kB) acc += partials[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(kB) k_lsqr_scalar(int stage, LsqrState* __restrict__ st,
                                                    const double* __restrict__ partials, int np) {
  __shared__ double sh[kB];
  if (st->done) return;
  const double val = block_sum(partials, np, sh);
  if (threadIdx.x != 0) return;
  LsqrState& S = *st;
  const double nrm = sqrt(val);
  switch (stage) {
    case kInitBeta:
      S.beta = nrm;
      S.bnorm = nrm;
      S.inv_beta = nrm > 0 ? 1.0 / nrm : 0.0;
      S.anorm2 = 0.0;
      S.itn = 0;
      S.istop = 0;
      S.rnorm = nrm;
      if (nrm == 0.0) {
        S.istop = 1;  // b = 0: x = 0 solves it exactly
        S.done = 1;
      }
      break;
    case kInitAlpha:
      S.alpha = nrm;
      S.inv_alpha = nrm > 0 ? 1.0 / nrm : 0.0;
      S.rhobar = nrm;
      S.phibar = S.beta;
      S.arnorm = nrm * S.beta;
      if (nrm == 0.0) {
        S.istop = 2;  // A^T b = 0: x = 0 is a least-squares solution
        S.done = 1;
      }
      break;
    case kBeta:
      S.beta = nrm;
      S.inv_beta = nrm > 0 ? 1.0 / nrm : 0.0;
      S.anorm2 += S.alpha * S.alpha + S.beta * S.beta;
      break;
    case kAlpha: {
      const double alpha = nrm;
      const double rho = hypot(S.rhobar, S.beta);
      const double c = S.rhobar / rho, s = S.beta / rho;
      const double theta = s * alpha;
      S.rhobar = -c * alpha;
      const double phi = c * S.phibar;
      S.phibar = s * S.phibar;
      S.rho = rho;
      S.phi = phi;
      S.theta = theta;
      S.cx = phi / rho;
      S.cw = theta / rho;
      S.rnorm = S.phibar;
      S.arnorm = S.phibar * alpha * fabs(c);
      S.alpha = alpha;
      S.inv_alpha = alpha > 0 ? 1.0 / alpha : 0.0;
      break;
    }
    case kXnorm: {
      S.xnorm2 = val;
      S.itn += 1;
      const double anorm = sqrt(S.anorm2);
      const double xnorm = nrm;
      if (S.rnorm <= S.tol * S.bnorm + S.tol * anorm * xnorm) {
        S.istop = 1;
        S.done = 1;
      } else if (S.arnorm <= S.tol * anorm * S.rnorm) {
        S.istop = 2;
        S.done = 1;
      } else if (S.itn >= S.maxit) {
        S.istop = 0;
        S.done = 1;
      }
      break;
    }
  }
}

__global__ void k_lsqr_reset(LsqrState* st, double tol, int maxit) {
  if (threadIdx.x == 0) {
    LsqrState S{};
    S.tol = tol;
    S.maxit = maxit;
    *st = S;
  }
}

// u~ = rhs, partial ||u~||^2
__global__ void __launch_bounds__(kB) k_copy_norm(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                                                  double* __restrict__ partial) {
  __shared__ double sh[kB];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    const double v = src[i];
    dst[i] = v;
    acc += v * v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// w = v~ / alpha, x = 0
__global__ void __launch_bounds__(kB) k_lsqr_init_xw(const LsqrState* __restrict__ st, const double* __restrict__ vt,
                                                     double* __restrict__ x, double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  x[i] = 0.0;
  w[i] = vt[i] * st->inv_alpha;
}

// x += cx w ; w = v~/alpha - cw w ; partial ||x||^2
__global__ void __launch_bounds__(kB) k_lsqr_update(const LsqrState* __restrict__ st, const double* __restrict__ vt,
                                                    double* __restrict__ x, double* __restrict__ w, int64_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[kB];
  if (st->done) return;
  const double cx = st->cx, cw = st->cw, ia = st->inv_alpha;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    const double wi = w[i];
    const double xi = x[i] + cx * wi;
    x[i] = xi;
    w[i] = vt[i] * ia - cw * wi;
    acc += xi * xi;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// ---------------------------------------------------------------------------
// vector kernels of the Newton drivers
// ---------------------------------------------------------------------------

// y = a * x + y
__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// y = a * x
__global__ void k_scale_copy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}

// out = -D * F
__global__ void k_neg_mul(int64_t n, const double* __restrict__ D, const double* __restrict__ F,
                          double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) out[i] = D ? -(D[i] * F[i]) : -F[i];
}

// partial sum of (D (a - b))^2, D optional
__global__ void __launch_bounds__(kB) k_diff_norm(int64_t n, const double* __restrict__ a, const double* __restrict__ b,
                                                  const double* __restrict__ D, double* __restrict__ partial) {
  __shared__ double sh[kB];
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    double d = a[i] - (b ? b[i] : 0.0);
    if (D) d *= D[i];
    acc += d * d;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

int vec_blocks(int64_t n) { return (int)std::min<int64_t>(std::max<int64_t>((n + kB - 1) / kB, 1), 1024); }

}  // namespace

void launch_axpy(Problem& P, int64_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_axpy, dim3((unsigned)((n + kB - 1) / kB)), dim3(kB), 0, P.stream, n, a, x, y);
  RFM_HIP(hipGetLastError());
}

void launch_scale_copy(Problem& P, int64_t n, double a, const double* x, double* y) {
  hipLaunchKernelGGL(k_scale_copy, dim3((unsigned)((n + kB - 1) / kB)), dim3(kB), 0, P.stream, n, a, x, y);
  RFM_HIP(hipGetLastError());
}

void launch_neg_mul(Problem& P, int64_t n, const double* D, const double* F, double* out) {
  hipLaunchKernelGGL(k_neg_mul, dim3((unsigned)((n + kB - 1) / kB)), dim3(kB), 0, P.stream, n, D, F, out);
  RFM_HIP(hipGetLastError());
}

// sum of (D (a - b))^2 into out[0]
void launch_diff_norm2(Problem& P, int64_t n, const double* a, const double* b, const double* D, double* out) {
  const int nb = vec_blocks(n);
  hipLaunchKernelGGL(k_diff_norm, dim3(nb), dim3(kB), 0, P.stream, n, a, b, D, P.d_red.p);
  launch_reduce_sum(P, P.d_red.p, nb, out);
}

// y [n] from min || (D J) R^{-1} y - rhs ||, rhs [m] on the device
void lsqr_run(Problem& P, const double* rhs, double tol, int maxit, double* y, int* iters, int* istop, int prec) {
  const int64_t m = P.m, n = P.n;
  RFM_CHECK(prec == RFM_PREC_F64 || (prec == RFM_PREC_F32 && P.have_J32), RFM_EINVAL,
            "LSQR: the FP32 Jacobian copy has not been formed");
  const bool f32 = prec == RFM_PREC_F32;
  auto jmul = [&](const double* x, double* yy, const double* up, double* part) {
    if (f32)
      launch_jmul(P, P.d_J32.p, x, yy, up, P.d_lsqr.p, part);
    else
      launch_jmul(P, P.d_J.p, x, yy, up, P.d_lsqr.p, part);
  };
  auto jtmul = [&](const double* yy, double* x) {
    if (f32)
      launch_jtmul(P, P.d_J32.p, yy, x, P.d_lsqr.p);
    else
      launch_jtmul(P, P.d_J.p, yy, x, P.d_lsqr.p);
  };
  const int nbk = (int)((n + trsv_block() - 1) / trsv_block());
  DBuf<double>& W = P.d_ws_lsqr;
  W.resize((size_t)m + 4 * (size_t)n + 3 * 65536);
  double* ut = W.p;
  double* vt = ut + m;
  double* w = vt + n;
  double* p = w + n;
  double* q = p + n;
  double* red_u = q + n;
  double* red_v = red_u + 65536;
  double* red_x = red_v + 65536;
  RFM_CHECK(P.ntiles <= 65536 && nbk <= 65536, RFM_EINVAL, "LSQR: too many reduction partials");
  LsqrState* st = P.d_lsqr.p;
  const int nbm = vec_blocks(m), nbn = vec_blocks(n);
  const unsigned gn = (unsigned)((n + kB - 1) / kB);

  hipLaunchKernelGGL(k_lsqr_reset, dim3(1), dim3(64), 0, P.stream, st, tol, maxit);
  // beta u = b
  hipLaunchKernelGGL(k_copy_norm, dim3(nbm), dim3(kB), 0, P.stream, rhs, ut, m, red_u);
  hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(kB), 0, P.stream, (int)kInitBeta, st, red_u, nbm);
  // alpha v = A^T u = R^{-T} (D J)^T (u~ / beta)
  jtmul(ut, q);
  launch_trsv(P, q, vt, true, nullptr, st, 0, 0, red_v);
  hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(kB), 0, P.stream, (int)kInitAlpha, st, red_v, nbk);
  hipLaunchKernelGGL(k_lsqr_init_xw, dim3(gn), dim3(kB), 0, P.stream, st, vt, y, w, n);
  RFM_HIP(hipGetLastError());

  ProfScope ps_all(P.prof, P.stream, "lsqr_total", 0.0, 0.0);
  const int poll = 8;
  int32_t done = 0;
  for (int it = 0; it < maxit && !done; ++it) {
    launch_trsv(P, vt, p, false, nullptr, st, 1, 0, nullptr);                 // p = R^{-1} v
    jmul(p, ut, ut, red_u);                                                    // u~ = A v - alpha u
    hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(kB), 0, P.stream, (int)kBeta, st, red_u, P.ntiles);
    jtmul(ut, q);                                                              // q = (D J)^T u
    launch_trsv(P, q, vt, true, vt, st, 0, 1, red_v);                          // v~ = R^{-T} q - beta v
    hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(kB), 0, P.stream, (int)kAlpha, st, red_v, nbk);
    hipLaunchKernelGGL(k_lsqr_update, dim3(nbn), dim3(kB), 0, P.stream, st, vt, y, w, n, red_x);
    hipLaunchKernelGGL(k_lsqr_scalar, dim3(1), dim3(kB), 0, P.stream, (int)kXnorm, st, red_x, nbn);
    RFM_HIP(hipGetLastError());
    if ((it + 1) % poll == 0 || it + 1 == maxit) {
      RFM_HIP(hipMemcpyAsync(&done, &st->done, sizeof(int32_t), hipMemcpyDeviceToHost, P.stream));
      RFM_HIP(hipStreamSynchronize(P.stream));
    }
  }
  LsqrState S;
  RFM_HIP(hipMemcpyAsync(&S, st, sizeof(S), hipMemcpyDeviceToHost, P.stream));
  RFM_HIP(hipStreamSynchronize(P.stream));
  check_trsv_error(P);
  *iters = S.itn;
  *istop = S.istop;
}

}  // namespace rfm
