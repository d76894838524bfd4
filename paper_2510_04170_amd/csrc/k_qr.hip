// Thin Householder QR of the sketch B (s x n, column-major, leading dimension s):
// the right preconditioner R of Alg. 1 step 2.  Only R is kept; Q is applied to
// the trailing columns as it is built and then dropped.
//
// Blocked right-looking algorithm with panels of ib <= 64 columns:
//  1. k_panel: one cooperative launch factors the panel column by column.  Each
//     workgroup keeps a contiguous chunk of the panel's rows in registers
//     (thread (rg, c) holds rows rg, rg+4, ... of column c).  A column costs one
//     grid barrier: the per-workgroup partial sums (sigma = ||x||^2 below the
//     diagonal and g_c = x^T a_c) are published, every workgroup reduces them in
//     the same fixed order and applies the reflector to its rows.  The reflector
//     follows the usual convention H = I - tau v v^T, v_0 = 1,
//     beta = -sign(alpha) ||(alpha, x)||.
//  2. The Gram V^T V (k_gemm_tn) and the compact-WY factor T (k_build_t), with
//     H_1 ... H_ib = I - V T V^T (Schreiber and Van Loan, 1989).
//  3. Trailing update C <- (I - V T^T V^T) C as W = V^T C (k_gemm_tn, split over
//     rows with a fixed-order reduction), W2 = -T^T W (k_reduce_w) and
//     C += V W2 (k_gemm_nn), both products on v_mfma_f64_16x16x4.
// Finally k_extract_r copies R (rows flipped to a positive diagonal) into the
// tiled upper storage used by the triangular solves and flags a zero or
// non-finite diagonal entry.
#include <algorithm>
#include <cmath>

#include "rfm_internal.h"

namespace rfm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kPanel = 64;      // panel width ib
constexpr int kTB = 64;         // tile size of the triangular-solve storage
constexpr int kSpinLimit = 1 << 26;

// sync words (d_sync): [0] grid barrier counter, [1] error flag, [2] singular flag
enum { kSyncBarrier = 0, kSyncError = 1, kSyncSingular = 2 };

__device__ __forceinline__ void grid_barrier(int32_t* sync, int nblocks, int& phase) {
  __syncthreads();
  ++phase;
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(&sync[kSyncBarrier], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    const int target = phase * nblocks;
    int spins = 0;
    while (__hip_atomic_load(&sync[kSyncBarrier], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if ((++spins & 1023) == 0 &&
          __hip_atomic_load(&sync[kSyncError], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
        break;  // another workgroup already gave up: drain
      if (spins > kSpinLimit) {
        __hip_atomic_store(&sync[kSyncError], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
    }
  }
  __syncthreads();
}

__global__ void k_reset_sync(int32_t* sync) {
  if (threadIdx.x == 0) sync[kSyncBarrier] = 0;
}

// Panel factorisation.  A: panel top-left (rows col0.., leading dimension ld),
// M rows, nb <= 64 columns; chunk rows per workgroup; RPT >= ceil(chunk / 4).
// P: partial-sum buffer [2][G][64], DR: diagonal-row buffer [2][64].
// Writes V below the diagonal and R on/above it in place, tau[nb], and the unit
// lower-trapezoidal V into Vb (M x 64, leading dimension ldv).
template <int RPT>
__global__ void __launch_bounds__(256) k_panel(double* __restrict__ A, int64_t ld, int M, int nb, int chunk,
                                               double* __restrict__ tau, double* __restrict__ P,
                                               double* __restrict__ DR, double* __restrict__ Vb, int64_t ldv,
                                               int32_t* __restrict__ sync) {
  __shared__ double colj[4][RPT];
  __shared__ double red[4][kPanel];
  __shared__ double scal_sh[4];
  const int G = gridDim.x, g = blockIdx.x;
  const int c = threadIdx.x % kPanel, rg = threadIdx.x / kPanel;
  const int r0 = g * chunk;
  const int rend = min(M, r0 + chunk);
  int phase = 0;

  double a[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int pr = r0 + rg + 4 * i;
    a[i] = (c < nb && pr < rend) ? A[(int64_t)c * ld + pr] : 0.0;
  }

  for (int j = 0; j < nb; ++j) {
    const int buf = j & 1;
    double* Pb = P + (size_t)buf * G * kPanel;
    double* DRb = DR + (size_t)buf * kPanel;
    // column j of this chunk to LDS
    if (c == j) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) colj[rg][i] = a[i];
    }
    __syncthreads();
    // partials over rows strictly below the diagonal
    double part = 0.0;
    if (c >= j && c < nb) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int pr = r0 + rg + 4 * i;
        if (pr > j && pr < rend) part += colj[rg][i] * a[i];
      }
    }
    red[rg][c] = part;
    // the diagonal row
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int pr = r0 + rg + 4 * i;
      if (pr == j && pr < rend && c >= j && c < nb) DRb[c] = a[i];  // only the owning chunk publishes
    }
    __syncthreads();
    if (rg == 0 && c >= j && c < nb) Pb[(size_t)g * kPanel + c] = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    grid_barrier(sync, G, phase);
    // reduce the partials of every workgroup in a fixed order
    double tot = 0.0;
    if (c >= j && c < nb) {
      for (int gg = rg; gg < G; gg += 4) tot += __builtin_nontemporal_load(&Pb[(size_t)gg * kPanel + c]);
    }
    red[rg][c] = tot;
    __syncthreads();
    double gc = (red[0][c] + red[1][c]) + (red[2][c] + red[3][c]);
    if (threadIdx.x == 0) {
      const double sigma = (red[0][j] + red[1][j]) + (red[2][j] + red[3][j]);
      const double alpha = __builtin_nontemporal_load(&DRb[j]);
      double beta, t, sc;
      if (sigma == 0.0) {
        beta = alpha;
        t = 0.0;
        sc = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + sigma), alpha);
        t = (beta - alpha) / beta;
        sc = 1.0 / (alpha - beta);
      }
      scal_sh[0] = beta;
      scal_sh[1] = t;
      scal_sh[2] = sc;
      if (g == 0) tau[j] = t;
    }
    __syncthreads();
    const double beta = scal_sh[0], t = scal_sh[1], sc = scal_sh[2];
    if (c > j && c < nb) {
      const double ajc = __builtin_nontemporal_load(&DRb[c]);
      const double wc = ajc + gc * sc;
      const double tw = t * wc;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int pr = r0 + rg + 4 * i;
        if (pr > j && pr < rend) a[i] -= tw * (colj[rg][i] * sc);
        else if (pr == j && pr < rend) a[i] -= tw;
      }
    } else if (c == j) {
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int pr = r0 + rg + 4 * i;
        if (pr > j && pr < rend) a[i] = colj[rg][i] * sc;
        else if (pr == j && pr < rend) a[i] = beta;
      }
    }
    __syncthreads();
  }
  // write back and emit the explicit V
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int pr = r0 + rg + 4 * i;
    if (pr < rend) {
      if (c < nb) A[(int64_t)c * ld + pr] = a[i];
      double v = 0.0;
      if (c < nb) v = pr > c ? a[i] : (pr == c ? 1.0 : 0.0);
      Vb[(int64_t)c * ldv + pr] = v;
    }
  }
}

// Split-row TN product: part[split][col][p] = sum_{k in split} V[k][p] C[k][col]
// V: K x 64 (ldv), C: K x N (ldc).  Workgroup tile 64 (p) x 64 (col); wavefront w
// owns p-tile w and the 4 col-tiles.  Rows are staged through LDS 32 at a time.
__global__ void __launch_bounds__(256) k_gemm_tn(const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ C, int64_t ldc, int K, int N,
                                                 int krange, double* __restrict__ part) {
  constexpr int KC = 32;
  __shared__ double Vs[KC][kPanel + 1];
  __shared__ double Cs[KC][kPanel + 1];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int n0 = blockIdx.x * 64;
  const int split = blockIdx.y;
  const int kb = split * krange, ke = min(K, kb + krange);
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) acc[ct] = v4d{0, 0, 0, 0};
  const int lk = tid % KC, lc = tid / KC;  // loader: row lk, columns lc + 8 i
  for (int k0 = kb; k0 < ke; k0 += KC) {
    const int kr = k0 + lk;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int col = lc + 8 * i;
      Vs[lk][col] = kr < ke ? V[(int64_t)col * ldv + kr] : 0.0;
      Cs[lk][col] = (kr < ke && n0 + col < N) ? C[(int64_t)(n0 + col) * ldc + kr] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < KC / 4; ++ks) {
      const int kk = ks * 4 + lane / 16;
      const double av = Vs[kk][wv * 16 + lane % 16];
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const double bv = Cs[kk][ct * 16 + lane % 16];
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // acc[ct][t]: p = wv*16 + (lane/16) + 4t, col = n0 + ct*16 + lane%16 (f64 MFMA result layout)
  double* o = part + (size_t)split * N * kPanel;
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int col = n0 + ct * 16 + lane % 16;
    if (col >= N) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) o[(int64_t)col * kPanel + wv * 16 + (lane / 16) + 4 * t] = acc[ct][t];
  }
}

// T of the compact-WY form from G = V^T V (summed over splits) and tau:
// T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j]   (columnwise, forward)
__global__ void __launch_bounds__(64) k_build_t(const double* __restrict__ part, int nsplit, int nb,
                                                const double* __restrict__ tau, double* __restrict__ T) {
  __shared__ double Ts[kPanel][kPanel + 1];
  __shared__ double Gj[kPanel];
  const int i = threadIdx.x;
  for (int r = 0; r < kPanel; ++r) Ts[r][i] = 0.0;
  __syncthreads();
  for (int j = 0; j < nb; ++j) {
    // column j of G: G[i][j] = sum_split part[split][j][i]
    double gij = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) gij += part[((size_t)sp * nb + j) * kPanel + i];
    Gj[i] = gij;
    __syncthreads();
    const double tj = tau[j];
    double v = 0.0;
    if (i < j) {
      for (int k = i; k < j; ++k) v += Ts[i][k] * Gj[k];
      v = -tj * v;
    } else if (i == j) {
      v = tj;
    }
    __syncthreads();
    if (i <= j) Ts[i][j] = v;
    __syncthreads();
  }
  for (int r = 0; r < kPanel; ++r) T[r * kPanel + i] = Ts[r][i];
}

// W2[col][p] = -sum_{q <= p} T[q][p] W[col][q], W = sum over splits
__global__ void __launch_bounds__(256) k_reduce_w(const double* __restrict__ part, int nsplit, int N,
                                                  const double* __restrict__ T, double* __restrict__ W2) {
  __shared__ double Wsh[4][kPanel];
  __shared__ double Tsh[kPanel][kPanel + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kPanel * kPanel; e += 256) Tsh[e / kPanel][e % kPanel] = T[e];
  const int p = tid % kPanel, sub = tid / kPanel;
  const int col = blockIdx.x * 4 + sub;
  double w = 0.0;
  if (col < N)
    for (int sp = 0; sp < nsplit; ++sp) w += part[((size_t)sp * N + col) * kPanel + p];
  Wsh[sub][p] = w;
  __syncthreads();
  if (col < N) {
    double v = 0.0;
    for (int q = 0; q <= p; ++q) v += Tsh[q][p] * Wsh[sub][q];
    W2[(int64_t)col * kPanel + p] = -v;
  }
}

// C[r][col] += sum_p V[r][p] W2[col][p]   (C: M x N, ldc; V: M x 64, ldv; W2: N x 64)
// workgroup tile 64 rows x 64 cols; wavefront w owns row tile w and 4 col tiles
__global__ void __launch_bounds__(256) k_gemm_nn(double* __restrict__ C, int64_t ldc,
                                                 const double* __restrict__ V, int64_t ldv,
                                                 const double* __restrict__ W2, int M, int N, int nb) {
  __shared__ double Ws[64][kPanel + 1];  // [col][p]
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int r0 = blockIdx.x * 64, n0 = blockIdx.y * 64;
  for (int e = tid; e < 64 * kPanel; e += 256) {
    const int col = e / kPanel, p = e % kPanel;
    Ws[col][p] = (n0 + col < N && p < nb) ? W2[(int64_t)(n0 + col) * kPanel + p] : 0.0;
  }
  __syncthreads();
  const int rbase = r0 + wv * 16;
  v4d acc[4];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int col = n0 + ct * 16 + lane % 16;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = rbase + (lane / 16) + 4 * t;
      acc[ct][t] = (r < M && col < N) ? C[(int64_t)col * ldc + r] : 0.0;
    }
  }
  const int nks = (nb + 3) / 4;
  for (int ks = 0; ks < nks; ++ks) {
    const int p = ks * 4 + lane / 16;
    const int r = rbase + lane % 16;
    const double av = (r < M && p < nb) ? V[(int64_t)p * ldv + r] : 0.0;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const double bv = Ws[ct * 16 + lane % 16][p];
      acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[ct], 0, 0, 0);
    }
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const int col = n0 + ct * 16 + lane % 16;
    if (col >= N) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int r = rbase + (lane / 16) + 4 * t;
      if (r < M) C[(int64_t)col * ldc + r] = acc[ct][t];
    }
  }
}

// R (upper n x n of B) into tiled storage: tile (bi, bj), bi <= bj, at
// ((bj (bj + 1)) / 2 + bi) * 64 * 64, column-major inside the tile, zero padded;
// row i is negated when B[i][i] < 0 so that diag(R) > 0.
__global__ void __launch_bounds__(256) k_extract_r(const double* __restrict__ B, int64_t ld, int n,
                                                   double* __restrict__ Rt, int32_t* __restrict__ sync) {
  const int bj = blockIdx.x, bi = blockIdx.y;
  if (bi > bj) return;
  double* tile = Rt + ((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB;
  for (int e = threadIdx.x; e < kTB * kTB; e += 256) {
    const int cc = e / kTB, rr = e % kTB;
    const int i = bi * kTB + rr, jcol = bj * kTB + cc;
    double v = 0.0;
    if (i < n && jcol < n && i <= jcol) {
      const double d = B[(int64_t)i * ld + i];
      v = B[(int64_t)jcol * ld + i];
      if (d < 0.0) v = -v;
      if (i == jcol && !(fabs(v) > 0.0 && isfinite(v))) sync[kSyncSingular] = 1;
    } else if (i == jcol) {
      v = 1.0;  // padding rows/cols past n: identity keeps the padded solve trivial
    }
    tile[e] = v;
  }
}

// R columns [c0, c0 + ncols) as dense column-major [ncols][n]
__global__ void k_get_r_cols(const double* __restrict__ Rt, int n, int64_t c0, double* __restrict__ out) {
  const int64_t jj = blockIdx.x;
  const int64_t jcol = c0 + jj;
  const int bj = (int)(jcol / kTB), cc = (int)(jcol % kTB);
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = 0.0;
    if (i <= jcol) {
      const int bi = i / kTB, rr = i % kTB;
      v = Rt[((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB + (size_t)cc * kTB + rr];
    }
    out[jj * n + i] = v;
  }
}

int g_num_cus = 0;

int num_cus(int device) {
  if (g_num_cus == 0) {
    hipDeviceProp_t prop;
    RFM_HIP(hipGetDeviceProperties(&prop, device));
    g_num_cus = prop.multiProcessorCount;
  }
  return g_num_cus;
}

template <int RPT>
void launch_panel_t(Problem& P, dim3 grid, double* A, int64_t ld, int M, int nb, int chunk, double* tau, double* Pp,
                    double* DR, double* Vb, int64_t ldv) {
  int32_t* sync = P.d_sync.p;
  void* args[] = {&A, &ld, &M, &nb, &chunk, &tau, &Pp, &DR, &Vb, &ldv, &sync};
  int maxb = 0;
  RFM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&maxb, reinterpret_cast<const void*>(&k_panel<RPT>), 256, 0));
  RFM_CHECK((int64_t)maxb * num_cus(P.device) >= (int64_t)grid.x, RFM_EDEVICE,
            "QR panel: workgroups cannot all be resident");
  RFM_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_panel<RPT>), grid, dim3(256), args, 0,
                                     P.stream));
}

void launch_panel(Problem& P, double* A, int64_t ld, int M, int nb, double* tau, double* Pp, double* DR, double* Vb,
                  int64_t ldv) {
  const int ncu = num_cus(P.device);
  int G = std::max(1, std::min(ncu, (M + 63) / 64));
  int chunk = (M + G - 1) / G;
  const int need = (chunk + 3) / 4;
  hipLaunchKernelGGL(k_reset_sync, dim3(1), dim3(64), 0, P.stream, P.d_sync.p);
  dim3 grid(G);
  if (need <= 16) launch_panel_t<16>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 32) launch_panel_t<32>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 48) launch_panel_t<48>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 64) launch_panel_t<64>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 80) launch_panel_t<80>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 104) launch_panel_t<104>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else throw Error(RFM_EINVAL, "QR panel: too many rows per workgroup (sketch too tall)");
}

}  // namespace

void qr_factor(Problem& P) {
  const int64_t s = P.s, n = P.n;
  RFM_CHECK(s >= n, RFM_EINVAL, "QR: sketch has fewer rows than columns");
  const int ncu = num_cus(P.device);
  // workspace: Vb (s x 64), T (64 x 64), P partials (2 x ncu x 64), DR (2 x 64),
  // TN partials (nsplit x max(N, 64) x 64), W2 (N x 64)
  const int max_split = 64;
  const size_t vb = (size_t)s * kPanel;
  const size_t tn = (size_t)max_split * std::max<int64_t>(n, kPanel) * kPanel;
  const size_t need = vb + kPanel * kPanel + 2 * (size_t)ncu * kPanel + 2 * kPanel + tn + (size_t)n * kPanel + 256;
  P.d_ws.resize(need);
  double* Vb = P.d_ws.p;
  double* T = Vb + vb;
  double* Pp = T + kPanel * kPanel;
  double* DR = Pp + 2 * (size_t)ncu * kPanel;
  double* part = DR + 2 * kPanel;
  double* W2 = part + tn;
  P.d_tau.resize(n);
  int32_t zero3[3] = {0, 0, 0};
  RFM_HIP(hipMemcpyAsync(P.d_sync.p, zero3, sizeof(zero3), hipMemcpyHostToDevice, P.stream));

  double* B = P.d_B.p;
  for (int64_t col0 = 0; col0 < n; col0 += kPanel) {
    const int nb = (int)std::min<int64_t>(kPanel, n - col0);
    const int M = (int)(s - col0);
    double* A = B + col0 * s + col0;
    launch_panel(P, A, s, M, nb, P.d_tau.p + col0, Pp, DR, Vb, M);
    // Gram V^T V with the same split-row product
    {
      int nsplit = std::min(max_split, std::max(1, M / 2048));
      int krange = ((M + nsplit - 1) / nsplit + 31) / 32 * 32;
      nsplit = (M + krange - 1) / krange;
      hipLaunchKernelGGL(k_gemm_tn, dim3(1, nsplit), dim3(256), 0, P.stream, Vb, (int64_t)M, Vb, (int64_t)M, M, nb,
                         krange, part);
      hipLaunchKernelGGL(k_build_t, dim3(1), dim3(64), 0, P.stream, part, nsplit, nb, P.d_tau.p + col0, T);
    }
    const int64_t N = n - col0 - nb;
    if (N > 0) {
      double* C = B + (col0 + nb) * s + col0;
      const int ntile = (int)((N + 63) / 64);
      int nsplit = std::max(1, std::min(max_split, (4 * ncu + ntile - 1) / ntile));
      nsplit = std::min<int>(nsplit, std::max(1, M / 256));
      int krange = ((M + nsplit - 1) / nsplit + 31) / 32 * 32;
      nsplit = (M + krange - 1) / krange;
      hipLaunchKernelGGL(k_gemm_tn, dim3(ntile, nsplit), dim3(256), 0, P.stream, Vb, (int64_t)M, C, s, M, (int)N,
                         krange, part);
      hipLaunchKernelGGL(k_reduce_w, dim3((unsigned)((N + 3) / 4)), dim3(256), 0, P.stream, part, nsplit, (int)N, T,
                         W2);
      hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((M + 63) / 64), (unsigned)ntile), dim3(256), 0, P.stream, C, s,
                         Vb, (int64_t)M, W2, M, (int)N, nb);
    }
    RFM_HIP(hipGetLastError());
  }
  // R to tiled storage
  const int nbt = (int)((n + kTB - 1) / kTB);
  P.d_R.resize((size_t)nbt * (nbt + 1) / 2 * kTB * kTB);
  hipLaunchKernelGGL(k_extract_r, dim3(nbt, nbt), dim3(256), 0, P.stream, B, s, (int)n, P.d_R.p, P.d_sync.p);
  RFM_HIP(hipGetLastError());
  int32_t flags[3];
  RFM_HIP(hipMemcpyAsync(flags, P.d_sync.p, sizeof(flags), hipMemcpyDeviceToHost, P.stream));
  RFM_HIP(hipStreamSynchronize(P.stream));
  RFM_CHECK(flags[kSyncError] == 0, RFM_EDEVICE, "QR panel: grid barrier timed out");
  RFM_CHECK(flags[kSyncSingular] == 0, RFM_ESINGULAR, "R has a zero or non-finite diagonal entry");
}

void launch_get_r_cols(Problem& P, int64_t c0, int64_t ncols, double* out) {
  hipLaunchKernelGGL(k_get_r_cols, dim3((unsigned)ncols), dim3(256), 0, P.stream, P.d_R.p, (int)P.n, c0, out);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
