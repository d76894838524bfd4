// Thin Householder QR of the sketch B (s x n, column-major, leading dimension s):
// the right preconditioner R of Alg. 1 step 2.  Only R is kept; Q is applied to
// the trailing columns as it is built and then dropped.
//
// Blocked right-looking algorithm with panels of ib <= 64 columns:
//  1. k_panel_df: one cooperative launch factors the panel column by column.  Each
//     workgroup keeps a contiguous chunk of the panel's rows in registers
//     (thread (rg, c) holds rows rg, rg+8, ... of column c).  Per column the
//     per-workgroup partial sums (sigma = ||x||^2 below the diagonal and
//     g_c = x^T a_c) are published in write-once slots, one owner workgroup per
//     column reduces them in a fixed order and publishes the total, and every
//     workgroup then applies the reflector to its rows (no grid barrier: readers
//     poll the slots; k_panel, with barriers, remains for panels with fewer rows
//     than columns).  The reflector follows the usual convention
//     H = I - tau v v^T, v_0 = 1, beta = -sign(alpha) ||(alpha, x)||.
//  2. The Gram V^T V (k_gemm_tn) and the compact-WY factor T (k_build_t), with
//     H_1 ... H_ib = I - V T V^T (Schreiber and Van Loan, 1989).
//  3. Inside a 256-column block, each 64-column block updates the rest of the
//     256 columns: W = V^T C (k_gemm_tn, split over rows with a fixed-order
//     reduction), W2 = -T^T W (k_reduce_w) and C += V W2 (k_gemm_nn), on
//     v_mfma_f64_16x16x4; the four T factors are merged into the block's T
//     (k_combine_t, then the 256-wide merge).
//  4. Outer panels are 512 columns: the first 256 are factored and applied to
//     the second 256 (K = 256), the second 256 are factored, the two T are
//     merged (T = [[Ta, -Ta Va^T Vb Tb], [0, Tb]]), and the trailing matrix is
//     updated once with K = 512 (k_gemm_tn128, k_reduce_wide, k_gemm_nn128 on
//     v_mfma_f64_4x4x4_4b), which halves the passes over it against K = 256.
// Finally k_extract_r copies R (rows flipped to a positive diagonal) into the
// tiled upper storage used by the triangular solves and flags a zero or
// non-finite diagonal entry.
#include <algorithm>
#include <chrono>
#include <functional>
#include <cmath>

#include "mfma_f64.h"
#include "rfm_internal.h"

namespace rfm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kPanel = 64;      // panel width ib
constexpr int kTB = 64;         // tile size of the triangular-solve storage
constexpr int kSpinLimit = 1 << 26;

// sync words (d_sync): [1] error flag, [2] singular flag, [1024, 1280) grid-barrier arrival words
enum { kSyncBarrier = 0, kSyncError = 1, kSyncSingular = 2, kSyncArrive = 1024 };

// Cross-workgroup exchange without cache maintenance: partial sums and the
// diagonal row are written and read with device-scope relaxed atomics (sc1,
// coherent across the XCDs' L2s); every wave waits for its stores to be
// acknowledged before the workgroup arrives at the barrier.
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// value of v in lane k (uniform k) for every lane of the wavefront
__device__ __forceinline__ double bcast_lane(double v, int k) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), k);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// sum over sp < cnt of p[sp * stride], added in split order (the loads go out 8 at a time; the sum is
// the same as one load and one add per split)
__device__ __forceinline__ double sum_splits(const double* __restrict__ p, size_t stride, int cnt) {
  double g = 0.0;
  int sp = 0;
  for (; sp + 8 <= cnt; sp += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = p[(size_t)(sp + q) * stride];
#pragma unroll
    for (int q = 0; q < 8; ++q) g += v[q];
  }
  for (; sp < cnt; ++sp) g += p[(size_t)sp * stride];
  return g;
}

// Grid barrier without atomics: workgroup g publishes its phase in its own word
// (after its data stores are acknowledged); thread t < G polls word t.  Arrival
// words start at 0 for every launch (k_reset_sync).
__device__ __forceinline__ void grid_barrier(int32_t* sync, int nblocks, int& phase) {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __syncthreads();
  ++phase;
  int32_t* arrive = sync + kSyncArrive;
  if (threadIdx.x == 0) __hip_atomic_store(&arrive[blockIdx.x], phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if ((int)threadIdx.x < nblocks) {
    int spins = 0;
    while (__hip_atomic_load(&arrive[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < phase) {
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
  sync[kSyncArrive + threadIdx.x] = 0;  // one word per workgroup, 256 threads
}

// Panel factorisation.  A: panel top-left (rows col0.., leading dimension ld),
// M rows, nb <= 64 columns; chunk rows per workgroup; RPT >= ceil(chunk / 8).
// P: partial-sum buffer [2][G][64] (G <= 256), DR: diagonal rows [2][64] then column totals [2][64].
// Writes V below the diagonal and R on/above it in place, tau[nb], and the unit
// lower-trapezoidal V into Vb (M x 64, leading dimension ldv).
// Thread (rg, c), rg < 8, holds rows rg, rg + 8, ... of column c of its chunk, so wavefront rg
// holds whole rows and lane j holds column j: the entries x_i of column j reach the other lanes
// by readlane, and the row tests (above, at or below row j) are uniform in the wavefront.  Per
// column j: partial sums x^T a_c below the diagonal, a grid-wide fixed-order reduction, then
// a_c -= tau w_c v with the Householder vector v (1 at row j, x sc below).
// ONE_BARRIER: every workgroup sums all partials itself (loads first, then a fixed-order sum);
// otherwise one workgroup per column sums them, publishes the total, and a second barrier follows.
template <int RPT, bool ONE_BARRIER>
__global__ void __launch_bounds__(512) k_panel(double* __restrict__ A, int64_t ld, int M, int nb, int chunk,
                                               double* __restrict__ tau, double* __restrict__ P,
                                               double* __restrict__ DR, double* __restrict__ Vb, int64_t ldv,
                                               int32_t* __restrict__ sync) {
  constexpr int NRG = 8;
  __shared__ double red[NRG][kPanel];
  __shared__ double scal_sh[4];
  __shared__ double sa_sh[2];
  const int G = gridDim.x, g = blockIdx.x;
  const int c = threadIdx.x % kPanel, rg = __builtin_amdgcn_readfirstlane(threadIdx.x / kPanel);  // uniform
  const int r0 = g * chunk;
  const int rend = min(M, r0 + chunk);
  int phase = 0;

  // this wavefront's row i is r0 + rg + 8 i, a row of the chunk for i < nrow (uniform)
  const int nrow = max(0, min(RPT, (rend - r0 - rg + NRG - 1) / NRG));
  double a[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) a[i] = (c < nb && i < nrow) ? A[(int64_t)c * ld + r0 + rg + NRG * i] : 0.0;

  for (int j = 0; j < nb; ++j) {
    const int buf = j & 1;
    double* Pb = P + (size_t)buf * G * kPanel;
    double* DRb = DR + (size_t)buf * kPanel;
    double* TOTb = DR + (size_t)(2 + buf) * kPanel;
    // rows below row j from i = ilo on, row j itself at i = idiag (or nowhere): uniform, so the
    // row tests are scalar compares against constants
    const int dj = j - r0 - rg;
    const int ilo = dj < 0 ? 0 : dj / NRG + 1;
    const int idiag = (dj >= 0 && dj % NRG == 0 && dj / NRG < nrow) ? dj / NRG : -1;
    // the diagonal row, published by the wavefront that holds it
    if (idiag >= 0 && c >= j && c < nb) {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == idiag) st_dev(&DRb[c], a[i]);
    }
    // partial sums over the rows below the diagonal (rows past the chunk hold 0)
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (i >= ilo) part += bcast_lane(a[i], j) * a[i];
    red[rg][c] = part;
    __syncthreads();
    if (rg == 0 && c >= j && c < nb)
      st_dev(&Pb[(size_t)g * kPanel + c], ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) +
                                              ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c])));
    grid_barrier(sync, G, phase);
    double gc = 0.0, ajc = 0.0;
    if (ONE_BARRIER) {
      // partials of workgroups rg, rg + 8, ... (G <= 256): all loads in flight, then the sums
      if (c >= j && c < nb) {
        double v[32];
#pragma unroll
        for (int k = 0; k < 32; ++k) {
          const int gg = rg + NRG * k;
          v[k] = gg < G ? ld_dev(&Pb[(size_t)gg * kPanel + c]) : 0.0;
        }
        ajc = ld_dev(&DRb[c]);
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int k = 0; k < 32; k += 2) {
          s0 += v[k];
          s1 += v[k + 1];
        }
        gc = s0 + s1;
      }
      red[rg][c] = gc;
      __syncthreads();
      gc = ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) + ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c]));
    } else {
      // workgroup g sums columns j + g, j + g + G, ... in a fixed order and publishes the totals
      for (int cc = g; cc < nb - j; cc += G) {
        const int col = j + cc;
        double v = (int)threadIdx.x < G ? ld_dev(&Pb[(size_t)threadIdx.x * kPanel + col]) : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6][0] = v;
        __syncthreads();
        if (threadIdx.x == 0)
          st_dev(&TOTb[col], ((red[0][0] + red[1][0]) + (red[2][0] + red[3][0])) +
                                 ((red[4][0] + red[5][0]) + (red[6][0] + red[7][0])));
        __syncthreads();
      }
      grid_barrier(sync, G, phase);
      if (c >= j && c < nb) {
        gc = ld_dev(&TOTb[c]);
        ajc = ld_dev(&DRb[c]);
      }
    }
    if (threadIdx.x == j) {
      sa_sh[0] = gc;   // sigma
      sa_sh[1] = ajc;  // alpha
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double sigma = sa_sh[0];
      const double alpha = sa_sh[1];
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
    // a_c -= tau w_c v for c > j; column j itself becomes (beta, v).  The empty asm keeps the
    // compiler from carrying the partial phase's broadcasts of column j over the barrier in SGPRs.
#pragma unroll
    for (int i = 0; i < RPT; ++i) asm volatile("" : "+v"(a[i]));
    const double tw = t * (ajc + gc * sc);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (i >= ilo) {
        const double v = bcast_lane(a[i], j) * sc;
        if (c == j) a[i] = v;
        else if (c > j) a[i] -= tw * v;
      } else if (i == idiag) {
        if (c == j) a[i] = beta;
        else if (c > j) a[i] -= tw;
      }
    }
    __syncthreads();
  }
  // write back and emit the explicit V
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    if (i < nrow) {
      const int pr = r0 + rg + NRG * i;
      if (c < nb) A[(int64_t)c * ld + pr] = a[i];
      double v = 0.0;
      if (c < nb) v = pr > c ? a[i] : (pr == c ? 1.0 : 0.0);
      Vb[(int64_t)c * ldv + pr] = v;
    }
  }
}

// Slots of the dataflow panel start every launch holding kEmpty, a signalling-NaN pattern: IEEE
// arithmetic only ever returns quiet NaNs, and every value published below is an arithmetic result
// (the diagonal row is canonicalised first), so a slot that differs from kEmpty holds its value.
constexpr unsigned long long kEmpty = 0xFFF4A5A5A5A5A5A5ull;

__global__ void k_fill_u64(unsigned long long* __restrict__ p, int64_t n, unsigned long long v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// the value of a published slot, polled until it is there (bounded: a time-out raises the error flag,
// and a raised flag ends every wait)
__device__ __forceinline__ double wait_slot(const double* p, int32_t* sync) {
  double v = ld_dev(p);
  int spins = 0;
  while ((unsigned long long)__double_as_longlong(v) == kEmpty) {
    __builtin_amdgcn_s_sleep(1);
    if ((++spins & 1023) == 0 &&
        __hip_atomic_load(&sync[kSyncError], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0)
      break;
    if (spins > kSpinLimit) {
      __hip_atomic_store(&sync[kSyncError], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      break;
    }
    v = ld_dev(p);
  }
  return v;
}

// Panel factorisation with the same arithmetic per column as k_panel and no grid barrier: every value
// that crosses workgroups sits in a slot of its own, written once per launch, and the readers poll it.
// Per column j: workgroup g publishes its partial sums x^T a_c (c >= j) in P[j][g][c] and, if it holds
// row j, the diagonal row in DR[j][c]; workgroup (c - j) mod G owns column c and sums the G partials
// of it in a fixed order into TOT[j][c]; every workgroup then reads TOT[j][c] and DR[j][c] and applies
// the reflector.  A reader depends only on writes that every workgroup makes before its first wait in
// the column, so all-resident workgroups cannot deadlock.  P: [64][G][64], DR: [64][64], TOT: [64][64],
// all kEmpty at launch.  Requires M >= nb (some workgroup holds every diagonal row).
template <int RPT>
__global__ void __launch_bounds__(512) k_panel_df(double* __restrict__ A, int64_t ld, int M, int nb, int chunk,
                                                  double* __restrict__ tau, double* __restrict__ P,
                                                  double* __restrict__ DR, double* __restrict__ TOT,
                                                  double* __restrict__ Vb, int64_t ldv, int32_t* __restrict__ sync) {
  constexpr int NRG = 8;
  __shared__ double red[NRG][kPanel];
  __shared__ double ored[NRG];
  __shared__ double tot_sh[kPanel], dr_sh[kPanel];
  __shared__ double scal_sh[3];
  const int G = gridDim.x, g = blockIdx.x;
  const int c = threadIdx.x % kPanel, rg = __builtin_amdgcn_readfirstlane(threadIdx.x / kPanel);  // uniform
  const int r0 = g * chunk;
  const int rend = min(M, r0 + chunk);
  const int nrow = max(0, min(RPT, (rend - r0 - rg + NRG - 1) / NRG));
  double a[RPT];
#pragma unroll
  for (int i = 0; i < RPT; ++i) a[i] = (c < nb && i < nrow) ? A[(int64_t)c * ld + r0 + rg + NRG * i] : 0.0;

  for (int j = 0; j < nb; ++j) {
    const int dj = j - r0 - rg;
    const int ilo = dj < 0 ? 0 : dj / NRG + 1;
    const int idiag = (dj >= 0 && dj % NRG == 0 && dj / NRG < nrow) ? dj / NRG : -1;
    if (idiag >= 0 && c >= j && c < nb) {
#pragma unroll
      for (int i = 0; i < RPT; ++i)
        if (i == idiag) st_dev(&DR[j * kPanel + c], __builtin_canonicalize(a[i]));
    }
    double part = 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i)
      if (i >= ilo) part += bcast_lane(a[i], j) * a[i];
    red[rg][c] = part;
    __syncthreads();
    if (rg == 0 && c >= j && c < nb)
      st_dev(&P[((size_t)j * G + g) * kPanel + c], ((red[0][c] + red[1][c]) + (red[2][c] + red[3][c])) +
                                                       ((red[4][c] + red[5][c]) + (red[6][c] + red[7][c])));
    // the columns this workgroup owns: partials of workgroups 0 .. G-1 in thread order
    for (int cc = g; cc < nb - j; cc += G) {
      const int col = j + cc;
      double v = (int)threadIdx.x < G ? wait_slot(&P[((size_t)j * G + threadIdx.x) * kPanel + col], sync) : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if ((threadIdx.x & 63) == 0) ored[threadIdx.x >> 6] = v;
      __syncthreads();
      if (threadIdx.x == 0)
        st_dev(&TOT[j * kPanel + col], ((ored[0] + ored[1]) + (ored[2] + ored[3])) + ((ored[4] + ored[5]) + (ored[6] + ored[7])));
      __syncthreads();
    }
    if (rg == 0 && c >= j && c < nb) {
      // both loads in flight at once (the diagonal row is usually there long before the total)
      double t = ld_dev(&TOT[j * kPanel + c]);
      double d = ld_dev(&DR[j * kPanel + c]);
      if ((unsigned long long)__double_as_longlong(t) == kEmpty) t = wait_slot(&TOT[j * kPanel + c], sync);
      if ((unsigned long long)__double_as_longlong(d) == kEmpty) d = wait_slot(&DR[j * kPanel + c], sync);
      tot_sh[c] = t;
      dr_sh[c] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double sigma = tot_sh[j];
      const double alpha = dr_sh[j];
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
    const double gc = (c >= j && c < nb) ? tot_sh[c] : 0.0;
    const double ajc = (c >= j && c < nb) ? dr_sh[c] : 0.0;
#pragma unroll
    for (int i = 0; i < RPT; ++i) asm volatile("" : "+v"(a[i]));
    const double tw = t * (ajc + gc * sc);
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      if (i >= ilo) {
        const double v = bcast_lane(a[i], j) * sc;
        if (c == j) a[i] = v;
        else if (c > j) a[i] -= tw * v;
      } else if (i == idiag) {
        if (c == j) a[i] = beta;
        else if (c > j) a[i] -= tw;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    if (i < nrow) {
      const int pr = r0 + rg + NRG * i;
      if (c < nb) A[(int64_t)c * ld + pr] = a[i];
      double v = 0.0;
      if (c < nb) v = pr > c ? a[i] : (pr == c ? 1.0 : 0.0);
      Vb[(int64_t)c * ldv + pr] = v;
    }
  }
}

// Split-row TN product: part[split][col][p] = sum_{k in split} V[k][p] C[k][col]
// V: K x 64 (ldv), C: K x N (ldc).  Workgroup tile 64 (p) x 64 (col); wavefront w
// owns p-tile w and the 4 col-tiles.  Rows are staged through LDS 32 at a time; the next 32 rows
// are loaded into registers while the current ones are multiplied.
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
  double rv[8], rcv[8];
  auto load = [&](int k0) {
    const int kr = k0 + lk;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int col = lc + 8 * i;
      rv[i] = kr < ke ? V[(int64_t)col * ldv + kr] : 0.0;
      rcv[i] = (kr < ke && n0 + col < N) ? C[(int64_t)(n0 + col) * ldc + kr] : 0.0;
    }
  };
  if (kb < ke) load(kb);
  for (int k0 = kb; k0 < ke; k0 += KC) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      Vs[lk][lc + 8 * i] = rv[i];
      Cs[lk][lc + 8 * i] = rcv[i];
    }
    __syncthreads();
    if (k0 + KC < ke) load(k0 + KC);
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
__global__ void __launch_bounds__(256) k_build_t(const double* __restrict__ part, int nsplit, int nb,
                                                 const double* __restrict__ tau, double* __restrict__ T) {
  __shared__ double Ts[kPanel][kPanel + 1];
  __shared__ double Gs[kPanel][kPanel + 1];  // Gs[j][i] = G[i][j]
  __shared__ double taus[kPanel];
  const int tid = threadIdx.x;
  for (int e = tid; e < kPanel * kPanel; e += 256) {
    const int j = e / kPanel, i = e % kPanel;
    double g = 0.0;
    if (j < nb)
      for (int sp = 0; sp < nsplit; ++sp) g += part[((size_t)sp * nb + j) * kPanel + i];
    Gs[j][i] = g;
    Ts[i][j] = 0.0;
  }
  if (tid < kPanel) taus[tid] = tid < nb ? tau[tid] : 0.0;
  __syncthreads();
  if (tid < kPanel) {
    // column j: T[i][j] = -tau_j sum_{i <= k < j} T[i][k] G[k][j], T[j][j] = tau_j (tau from LDS: one
    // global load per column would put a memory round trip on every step of this chain)
    const int i = tid;
    for (int j = 0; j < nb; ++j) {
      const double tj = taus[j];
      double v = 0.0;
      if (i < j) {
        // in order of k, the LDS reads 8 at a time
        int k = i;
        for (; k + 8 <= j; k += 8) {
          double a[8], g[8];
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            a[q] = Ts[i][k + q];
            g[q] = Gs[j][k + q];
          }
#pragma unroll
          for (int q = 0; q < 8; ++q) v += a[q] * g[q];
        }
        for (; k < j; ++k) v += Ts[i][k] * Gs[j][k];
        v = -tj * v;
      } else if (i == j) {
        v = tj;
      }
      // every lane reads columns < j only; the write goes to column j
      if (i <= j) Ts[i][j] = v;
      __builtin_amdgcn_wave_barrier();
    }
  }
  __syncthreads();
  for (int e = tid; e < kPanel * kPanel; e += 256) T[e] = Ts[e / kPanel][e % kPanel];
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
  if (col < N) w = sum_splits(part + (size_t)col * kPanel + p, (size_t)N * kPanel, nsplit);
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
  // all of this lane's V values first (one memory round trip), then the products in order of p
  const int nks = (nb + 3) / 4;
  const int r = rbase + lane % 16;
  double avs[kPanel / 4];
#pragma unroll
  for (int ks = 0; ks < kPanel / 4; ++ks) {
    const int p = ks * 4 + lane / 16;
    avs[ks] = (ks < nks && r < M && p < nb) ? V[(int64_t)p * ldv + r] : 0.0;
  }
#pragma unroll
  for (int ks = 0; ks < kPanel / 4; ++ks) {
    if (ks < nks) {  // uniform
      const int p = ks * 4 + lane / 16;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const double bv = Ws[ct * 16 + lane % 16][p];
        acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(avs[ks], bv, acc[ct], 0, 0, 0);
      }
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

// ---------------------------------------------------------------------------
// 128 x 128 tiles for the trailing update of 256-column outer panels.
// Four wavefronts in a 2 x 2 arrangement each own a 64 x 64 block of 64
// accumulators per lane on v_mfma_f64_4x4x4_4b_f64 (measured on gfx950 at
// about 1.5x the FP64 rate of the 16x16x4 form).  Operands are staged through
// LDS 16 values of k at a time; the next chunk's global loads (16 bytes per
// lane) are issued before the current chunk's MFMAs.  The chunk routine and
// the XCD-aware workgroup order are in mfma_f64.h.
// ---------------------------------------------------------------------------

// C[M x N] += A[M x K] B, A column-major (lda even, base 16-byte aligned, lda >= M), B k-major
// (B[k][n] = Bk[k * ldbk + n], ldbk even, base aligned, ldbk >= N); K a multiple of 32.
// Operands move from global memory straight into LDS (global_load_lds_dwordx4): per 16-deep chunk each
// wavefront issues 4 k-rows of A and 4 of B, one 16-byte piece per lane, into tiles with rows of 130
// doubles; two tile pairs in separate LDS arrays, so the reads of one are not made to wait for the
// loads into the other, and one barrier per chunk.  Rows past M and columns past N load clamped
// (in-bounds) addresses and are never stored.
// 1-D grid over the tiles: each XCD takes a contiguous range of the tiles ordered in groups of 4 row
// tiles (row tile fastest), so the 4 x 4 tiles it runs at a time share 4 tiles of A and 4 of B in its L2
// (against a fresh A tile per workgroup in row-major launch order; 8% faster at K = 512).
typedef __attribute__((address_space(3))) void* lds_ptr;
constexpr int kLdsRow = kBig + 2;  // 16-byte aligned rows

__global__ void __launch_bounds__(256, 2) k_gemm_nn128(double* __restrict__ C, int64_t ldc,
                                                      const double* __restrict__ A, int64_t lda,
                                                      const double* __restrict__ Bk, int64_t ldbk, int M, int N,
                                                      int K) {
  __shared__ __attribute__((aligned(16))) double As0[kKC][kLdsRow];
  __shared__ __attribute__((aligned(16))) double Bs0[kKC][kLdsRow];
  __shared__ __attribute__((aligned(16))) double As1[kKC][kLdsRow];
  __shared__ __attribute__((aligned(16))) double Bs1[kKC][kLdsRow];
  const int tid = threadIdx.x, lane = tid % 64, wv = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wr = wv / 2, wc = wv % 2;
  int r0, n0;
  {
    constexpr int kGroup = 4;
    const int nrt = (M + kBig - 1) / kBig, nct = (N + kBig - 1) / kBig;
    const int L = xcd_order(blockIdx.x, nrt * nct);
    const int gi = L / (kGroup * nct), gl = L % (kGroup * nct);
    const int gh = min(kGroup, nrt - gi * kGroup);
    r0 = (gi * kGroup + gl % gh) * kBig;
    n0 = (gl / gh) * kBig;
  }
  double acc[4][16];
#pragma unroll
  for (int rg = 0; rg < 4; ++rg)
#pragma unroll
    for (int cg = 0; cg < 16; ++cg) acc[rg][cg] = 0.0;
  const int64_t ra = min<int64_t>(r0 + 2 * lane, lda - 2);
  const int64_t nbk = min<int64_t>(n0 + 2 * lane, ldbk - 2);
  auto issue = [&](int k0, double (*Xs)[kLdsRow], double (*Ys)[kLdsRow]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int kk = wv * 4 + i;
      __builtin_amdgcn_global_load_lds((const void*)(A + (int64_t)(k0 + kk) * lda + ra), (lds_ptr)&Xs[kk][0], 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(Bk + (int64_t)(k0 + kk) * ldbk + nbk), (lds_ptr)&Ys[kk][0], 16, 0,
                                       0);
    }
  };
  issue(0, As0, Bs0);
  for (int k0 = 0; k0 < K; k0 += 2 * kKC) {
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's pieces of the chunk have landed
    __syncthreads();                // everyone's have, and nobody still reads the other pair
    issue(k0 + kKC, As1, Bs1);
    mfma4_chunk(As0, Bs0, lane, wr, wc, acc);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (k0 + 2 * kKC < K) issue(k0 + 2 * kKC, As0, Bs0);
    mfma4_chunk(As1, Bs1, lane, wr, wc, acc);
  }
  // C += acc, two row groups (32 loads per lane) at a time
  const int row_l = lane % 16, col_l = lane / 16;
#pragma unroll
  for (int rp = 0; rp < 4; rp += 2) {
    double cv[2][16];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = r0 + wr * 64 + (rp + q) * 16 + row_l;
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) {
        const int col = n0 + wc * 64 + cg * 4 + col_l;
        cv[q][cg] = (col < N && r < M) ? C[(int64_t)col * ldc + r] : 0.0;
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int r = r0 + wr * 64 + (rp + q) * 16 + row_l;
#pragma unroll
      for (int cg = 0; cg < 16; ++cg) {
        const int col = n0 + wc * 64 + cg * 4 + col_l;
        if (col < N && r < M) C[(int64_t)col * ldc + r] = cv[q][cg] + acc[rp + q][cg];
      }
    }
  }
}

// Tiles of 128 (p or n) x 16 (k) for the TN product, staged as 16-byte pairs (k, k + 1): the pair of
// k-pair c of index p sits in slot p * 8 + (c ^ ((p / 2) % 8)).  Loading a column's 16 k is then one
// contiguous 128-byte piece spread over its 8 slots, and the 16 lanes of a wavefront that read one k of
// 16 consecutive p hit distinct LDS banks.
__device__ __forceinline__ int pair_slot(int p, int c) { return p * 8 + (c ^ ((p / 2) % 8)); }

// One 16-deep k-chunk on pair tiles Xp (output rows p) and Yp (output columns n); the same products, in
// the same order, as mfma4_chunk on plain tiles.
__device__ __forceinline__ void mfma4_chunk_pairs(const double* Xp, const double* Yp, int lane, int wr, int wc,
                                                  double (&acc)[4][16]) {
  const int h = lane / 32, odd = (lane / 16) % 2;  // k = 4 ks + lane / 16: pair 2 ks + h, element odd
  const int m = (lane % 16) / 2;
#pragma unroll
  for (int ks = 0; ks < kKC / 4; ++ks) {
    const int xoff = (lane % 16) * 16 + 2 * ((2 * ks) ^ (h ^ m)) + odd;
    double x[4];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) x[rg] = Xp[(wr * 64 + rg * 16) * 16 + xoff];
    const int yl = (lane % 4) * 16 + 2 * (h ^ ((lane % 4) / 2)) + odd;
#pragma unroll
    for (int hh = 0; hh < 2; ++hh) {
      double y[8];
#pragma unroll
      for (int cg = 0; cg < 8; ++cg) {
        const int cq = hh * 8 + cg;
        y[cg] = Yp[(wc * 64 + cq * 4) * 16 + 4 * (ks ^ (cq % 4)) + yl];
      }
#pragma unroll
      for (int rg = 0; rg < 4; ++rg)
#pragma unroll
        for (int cg = 0; cg < 8; ++cg)
          acc[rg][hh * 8 + cg] = __builtin_amdgcn_mfma_f64_4x4x4f64(y[cg], x[rg], acc[rg][hh * 8 + cg], 0, 0, 0);
    }
  }
}

// part[split][n][p] = sum_{k in split} A[k][p] B[k][n]; A: K x pstride (lda), B: K x N (ldb), both
// column-major; rows of a split: [split * krange, ...), krange a multiple of 16.  Grid: 1-D,
// (pstride / 128 halves) x (column tiles) x (row splits) workgroups.  Whole 16-row chunks move from
// global memory straight into the pair tiles (global_load_lds_dwordx4, one 16-byte pair per lane,
// columns past N clamped to N - 1 and never stored); a split's last, partial chunk, and every chunk
// when VEC is false, go through registers with guarded loads.  VEC: lda, ldb even and both bases 16-byte
// aligned.  GRAM only tells the Gram products of the T merges apart from the trailing updates in a
// profile (same code).
template <bool VEC, bool GRAM = false>
__global__ void __launch_bounds__(256, 2) k_gemm_tn128(const double* __restrict__ A, int64_t lda,
                                                     const double* __restrict__ B, int64_t ldb, int K, int N,
                                                     int krange, double* __restrict__ part, int pstride) {
  __shared__ __attribute__((aligned(16))) double Xp0[kBig * kKC];
  __shared__ __attribute__((aligned(16))) double Yp0[kBig * kKC];
  __shared__ __attribute__((aligned(16))) double Xp1[kBig * kKC];
  __shared__ __attribute__((aligned(16))) double Yp1[kBig * kKC];
  const int tid = threadIdx.x, lane = tid % 64, wv = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wr = wv / 2, wc = wv % 2;
  // 1-D grid of halves x column tiles x splits: on each XCD the halves of one (column tile, split)
  // run next to each other and share that C tile in its L2
  const int halves = pstride / kBig, ntile = (N + kBig - 1) / kBig;
  const int L = xcd_order(blockIdx.x, gridDim.x);
  const int half = L % halves;
  const int n0 = (L / halves) % ntile * kBig;
  const int split = L / halves / ntile;
  A += (int64_t)half * kBig * lda;
  const int kb = split * krange, ke = min(K, kb + krange);
  double acc[4][16];
#pragma unroll
  for (int rg = 0; rg < 4; ++rg)
#pragma unroll
    for (int cg = 0; cg < 16; ++cg) acc[rg][cg] = 0.0;
  // direct loads: instruction b of a tile covers indices 8 b .. 8 b + 7, lane l index 8 b + l / 8, slot
  // l % 8; per-lane byte offsets from the tile's first column at the chunk's first row (32-bit: the host
  // keeps 128 ld 8 < 2^32)
  uint32_t ao[4], bo[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int p = (wv * 4 + i) * 8 + lane / 8;
    const int c = (lane % 8) ^ ((p / 2) % 8);
    ao[i] = (uint32_t)(((int64_t)p * lda + 2 * c) * 8);
    bo[i] = (uint32_t)(((int64_t)min(p, N - 1 - n0) * ldb + 2 * c) * 8);  // relative to column n0
  }
  auto issue = [&](int k0, double* Xs, double* Ys) {
    const char* ab = reinterpret_cast<const char*>(A + k0);
    const char* bb = reinterpret_cast<const char*>(B + (int64_t)n0 * ldb + k0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int blk = wv * 4 + i;
      __builtin_amdgcn_global_load_lds((const void*)(ab + ao[i]), (lds_ptr)(Xs + blk * 128), 16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(bb + bo[i]), (lds_ptr)(Ys + blk * 128), 16, 0, 0);
    }
  };
  // whole chunks by direct loads, two tile pairs, one barrier per chunk
  const int nfull = VEC && ke > kb ? (ke - kb) / kKC : 0;
  if (nfull > 0) issue(kb, Xp0, Yp0);
  for (int ch = 0; ch < nfull; ch += 2) {
    __builtin_amdgcn_s_waitcnt(0);  // this wavefront's pieces of the chunk have landed
    __syncthreads();                // everyone's have, and nobody still reads the other pair
    if (ch + 1 < nfull) issue(kb + (ch + 1) * kKC, Xp1, Yp1);
    mfma4_chunk_pairs(Xp0, Yp0, lane, wr, wc, acc);
    if (ch + 1 >= nfull) break;
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (ch + 2 < nfull) issue(kb + (ch + 2) * kKC, Xp0, Yp0);
    mfma4_chunk_pairs(Xp1, Yp1, lane, wr, wc, acc);
  }
  // the rest (a split's partial last chunk; every chunk when VEC is false) through registers with
  // guarded loads: thread t fills slots t + 256 i of both tiles
  for (int k0 = kb + nfull * kKC; k0 < ke; k0 += kKC) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int sl = tid + 256 * i;
      const int p = sl / 8;
      const int c = (sl % 8) ^ ((p / 2) % 8);
      const int k = k0 + 2 * c;
      const bool nv = n0 + p < N;
      const double* ap = A + (int64_t)p * lda + k;
      const double* bp = B + (int64_t)(n0 + p) * ldb + k;
      Xp0[2 * sl] = k < ke ? ap[0] : 0.0;
      Xp0[2 * sl + 1] = k + 1 < ke ? ap[1] : 0.0;
      Yp0[2 * sl] = (nv && k < ke) ? bp[0] : 0.0;
      Yp0[2 * sl + 1] = (nv && k + 1 < ke) ? bp[1] : 0.0;
    }
    __syncthreads();
    mfma4_chunk_pairs(Xp0, Yp0, lane, wr, wc, acc);
  }
  double* o = part + (size_t)split * N * pstride + (size_t)half * kBig;
  const int row_l = lane % 16, col_l = lane / 16;
#pragma unroll
  for (int cg = 0; cg < 16; ++cg) {
    const int col = n0 + wc * 64 + cg * 4 + col_l;
    if (col >= N) continue;
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) o[(int64_t)col * pstride + wr * 64 + rg * 16 + row_l] = acc[rg][cg];
  }
}

// W2[n][p] = -sum_{q <= p} T[q][p] W[n][q], W = sum over splits of part (T: 128 x 128 row-major)
__global__ void __launch_bounds__(256) k_reduce_w128(const double* __restrict__ part, int nsplit, int N,
                                                     const double* __restrict__ T, double* __restrict__ W2) {
  __shared__ double Wsh[2][kBig];
  const int p = threadIdx.x % kBig, sub = threadIdx.x / kBig;
  const int n = blockIdx.x * 2 + sub;
  double w = 0.0;
  if (n < N)
    for (int sp = 0; sp < nsplit; ++sp) w += part[((size_t)sp * N + n) * kBig + p];
  Wsh[sub][p] = w;
  __syncthreads();
  if (n < N) {
    double v = 0.0;
    for (int qq = 0; qq <= p; ++qq) v += T[qq * kBig + p] * Wsh[sub][qq];
    W2[(int64_t)n * kBig + p] = -v;
  }
}

// T (128 x 128, row-major) of two consecutive 64-column reflector blocks:
// [[Ta, -Ta Gab Tb], [0, Tb]], Gab = Va^T Vb from split partials part[split][b][a]
__global__ void __launch_bounds__(256) k_combine_t(const double* __restrict__ Ta, const double* __restrict__ Tb,
                                                   const double* __restrict__ part, int nsplit, int nbb,
                                                   double* __restrict__ T) {
  __shared__ double Xs[kPanel][kPanel + 1];
  __shared__ double Gs[kPanel][kPanel + 1];
  __shared__ double Tas[kPanel][kPanel + 1];
  __shared__ double Tbs[kPanel][kPanel + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < kPanel * kPanel; e += 256) {
    const int a = e / kPanel, b = e % kPanel;
    double g = 0.0;
    if (b < nbb)
      for (int sp = 0; sp < nsplit; ++sp) g += part[((size_t)sp * nbb + b) * kPanel + a];
    Gs[a][b] = g;
    Tas[a][b] = Ta[e];
    Tbs[a][b] = Tb[e];
  }
  __syncthreads();
  // X = Gab Tb (Tb upper triangular)
  for (int e = tid; e < kPanel * kPanel; e += 256) {
    const int a = e / kPanel, b = e % kPanel;
    double v = 0.0;
    if (nbb > 0) {
      int k = 0;
      for (; k + 8 <= b + 1; k += 8) {
        double x[8], y[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          x[q] = Gs[a][k + q];
          y[q] = Tbs[k + q][b];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v += x[q] * y[q];
      }
      for (; k <= b; ++k) v += Gs[a][k] * Tbs[k][b];
    }
    Xs[a][b] = v;
  }
  __syncthreads();
  for (int e = tid; e < kBig * kBig; e += 256) {
    const int qq = e / kBig, p = e % kBig;
    double v = 0.0;
    if (qq < kPanel && p < kPanel) {
      v = Tas[qq][p];
    } else if (qq >= kPanel && p >= kPanel) {
      v = Tbs[qq - kPanel][p - kPanel];
    } else if (qq < kPanel && p >= kPanel) {
      const int b = p - kPanel;
      int k = qq;
      for (; k + 8 <= kPanel; k += 8) {
        double x[8], y[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          x[q] = Tas[qq][k + q];
          y[q] = Xs[k + q][b];
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) v += x[q] * y[q];
      }
      for (; k < kPanel; ++k) v += Tas[qq][k] * Xs[k][b];
      v = -v;
    }
    T[e] = v;
  }
}

// zero the top 64 rows of columns 64..127 of V (M x 128, leading dimension ldv)
__global__ void k_zero_top(double* __restrict__ V, int64_t ldv) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < kPanel * kPanel) V[(int64_t)(kPanel + e / kPanel) * ldv + e % kPanel] = 0.0;
}

// ---------------------------------------------------------------------------
// Outer panels: 256-column blocks (four 64-column reflector blocks) and the
// 512-column trailing-update width (two 256-column blocks); T of the merged
// blocks and the -T^T W reduction
// ---------------------------------------------------------------------------
constexpr int kOuter = 256;
constexpr int kWide = 512;

// zero rows [0, nrows) of columns [c0, c0 + ncols) of V (leading dimension ldv)
__global__ void k_zero_block(double* __restrict__ V, int64_t ldv, int c0, int ncols, int nrows) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)ncols * nrows) V[(int64_t)(c0 + e / nrows) * ldv + e % nrows] = 0.0;
}

__global__ void k_fill(double* __restrict__ p, int64_t n, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = v;
}

// G[b][a] = sum over splits of part[split][b][a] for b < nb (64-wide rows), splits in order; the
// single-workgroup T builders then read G as a one-split partial
// G[e] = sum over splits of part[split][e] in split order, e < nb * 64; the loads go out 8 at a time
__global__ void __launch_bounds__(256) k_gsum64(const double* __restrict__ part, int nsplit, int nb,
                                                double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int ne = nb * kPanel;
  if (e >= ne) return;
  G[e] = sum_splits(part + e, (size_t)ne, nsplit);
}

// G[a][b] (row-major w x w) = sum over splits of part[split][b][a] (pstride w), splits in order
__global__ void k_gsum(const double* __restrict__ part, int nsplit, int w, double* __restrict__ G) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w * w) return;
  const int a = e / w, b = e % w;
  G[e] = sum_splits(part + (size_t)b * w + a, (size_t)w * w, nsplit);
}

// C = alpha * A B for row-major w x w matrices, one thread per entry
__global__ void k_sq_gemm(const double* __restrict__ A, const double* __restrict__ B, double alpha, int w,
                          double* __restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= w * w) return;
  const int i = e / w, j = e % w;
  double v = 0.0;
  int k = 0;
  for (; k + 8 <= w; k += 8) {  // loads 8 at a time, the sum in order of k
    double a[8], b[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      a[q] = A[i * w + k + q];
      b[q] = B[(k + q) * w + j];
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) v += a[q] * b[q];
  }
  for (; k < w; ++k) v += A[i * w + k] * B[k * w + j];
  C[e] = alpha * v;
}

// T (2w x 2w, row-major) = [[T1, Y], [0, T2]] from w x w blocks
__global__ void k_assemble_t(const double* __restrict__ T1, const double* __restrict__ T2,
                             const double* __restrict__ Y, int w, double* __restrict__ T) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 4 * w * w) return;
  const int qq = e / (2 * w), p = e % (2 * w);
  double v = 0.0;
  if (qq < w && p < w) v = T1[qq * w + p];
  else if (qq >= w && p >= w) v = T2[(qq - w) * w + (p - w)];
  else if (qq < w && p >= w) v = Y[qq * w + (p - w)];
  T[e] = v;
}

// W2[p][n] = W2k[p * ldw + n] = -sum_{q <= p} T[q][p] W[n][q] for WID (256 or 512) reflectors, W = sum
// over splits (pstride WID); one thread per p, 8 columns per block.  W2 is k-major for the product
// C += V W2 (its rows are the k-rows that product loads).
template <int WID>
__global__ void __launch_bounds__(WID) k_reduce_wide(const double* __restrict__ part, int nsplit, int N,
                                                     const double* __restrict__ T, double* __restrict__ W2,
                                                     int64_t ldw) {
  __shared__ double Wsh[8][WID];
  const int p = threadIdx.x;
  const int n0 = blockIdx.x * 8;
  for (int c = 0; c < 8; ++c) {
    const int n = n0 + c;
    double w = 0.0;
    if (n < N) w = sum_splits(part + (size_t)n * WID + p, (size_t)N * WID, nsplit);
    Wsh[c][p] = w;
  }
  __syncthreads();
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int qq = 0;
  for (; qq + 8 <= p + 1; qq += 8) {  // T loads 8 at a time, the sums in order of qq
    double t[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = T[(qq + q) * WID + p];
#pragma unroll
    for (int q = 0; q < 8; ++q)
#pragma unroll
      for (int c = 0; c < 8; ++c) v[c] += t[q] * Wsh[c][qq + q];
  }
  for (; qq <= p; ++qq) {
    const double t = T[qq * WID + p];
#pragma unroll
    for (int c = 0; c < 8; ++c) v[c] += t * Wsh[c][qq];
  }
#pragma unroll
  for (int c = 0; c < 8; ++c)
    if (n0 + c < N) W2[(int64_t)p * ldw + n0 + c] = -v[c];
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

// Streamed QR: rows col0 .. col0 + 511 of the tiled R, columns col0 .. n - 1, into the slot rows
// 0 .. 511 of Y (column j at Y[j ldy + r]); zero below R's diagonal and past row n - 1.
__global__ void k_strip_in(const double* __restrict__ Rt, int n, int64_t col0, double* __restrict__ Y, int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t jcol = col0 + e / kWide;
  const int r = (int)(e % kWide);
  if (jcol >= n) return;
  const int64_t i = col0 + r;
  double v = 0.0;
  if (i < n && i <= jcol) {
    const int bi = (int)(i / kTB), bj = (int)(jcol / kTB);
    v = Rt[((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB + (size_t)(jcol % kTB) * kTB + i % kTB];
  }
  Y[jcol * ldy + r] = v;
}

// the slot rows back into R (on and above the diagonal)
__global__ void k_strip_out(double* __restrict__ Rt, int n, int64_t col0, const double* __restrict__ Y,
                            int64_t ldy) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t jcol = col0 + e / kWide;
  const int r = (int)(e % kWide);
  if (jcol >= n) return;
  const int64_t i = col0 + r;
  if (i < n && i <= jcol) {
    const int bi = (int)(i / kTB), bj = (int)(jcol / kTB);
    Rt[((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB + (size_t)(jcol % kTB) * kTB + i % kTB] = Y[jcol * ldy + r];
  }
}

// sign[i] = -1 where R[i][i] < 0, else 1; flags a zero or non-finite diagonal entry
__global__ void k_r_signs(const double* __restrict__ Rt, int n, double* __restrict__ sign, int32_t* __restrict__ sync) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int bi = i / kTB;
  const double d = Rt[((size_t)bi * (bi + 1) / 2 + bi) * kTB * kTB + (size_t)(i % kTB) * kTB + i % kTB];
  if (!(fabs(d) > 0.0 && isfinite(d))) sync[kSyncSingular] = 1;
  sign[i] = d < 0.0 ? -1.0 : 1.0;
}

// rows times their signs; the diagonal past n set to 1 (the padded solve stays trivial)
__global__ void __launch_bounds__(256) k_r_apply_signs(double* __restrict__ Rt, int n, const double* __restrict__ sign) {
  const int bj = blockIdx.x, bi = blockIdx.y;
  if (bi > bj) return;
  double* tile = Rt + ((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB;
  for (int e = threadIdx.x; e < kTB * kTB; e += 256) {
    const int cc = e / kTB, rr = e % kTB;
    const int i = bi * kTB + rr, jcol = bj * kTB + cc;
    if (i < n)
      tile[e] *= sign[i];
    else if (i == jcol)
      tile[e] = 1.0;
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

// one barrier per column (every workgroup reduces all partials) or two (one reducer per column)
constexpr bool kPanelOneBarrier = true;

template <int RPT>
void launch_panel_t(Problem& P, dim3 grid, double* A, int64_t ld, int M, int nb, int chunk, double* tau, double* Pp,
                    double* DR, double* Vb, int64_t ldv) {
  int32_t* sync = P.d_sync.p;
  const void* fn;
  if (M >= nb) {
    // dataflow form: P [64][G][64], then DR [64][64] and TOT [64][64], all set to kEmpty
    const int64_t cnt = (int64_t)kPanel * grid.x * kPanel;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, P.stream,
                       reinterpret_cast<unsigned long long*>(Pp), cnt, kEmpty);
    hipLaunchKernelGGL(k_fill_u64, dim3(2 * kPanel * kPanel / 256), dim3(256), 0, P.stream,
                       reinterpret_cast<unsigned long long*>(DR), (int64_t)2 * kPanel * kPanel, kEmpty);
    fn = reinterpret_cast<const void*>(&k_panel_df<RPT>);
  } else {
    hipLaunchKernelGGL(k_reset_sync, dim3(1), dim3(256), 0, P.stream, P.d_sync.p);
    fn = reinterpret_cast<const void*>(&k_panel<RPT, kPanelOneBarrier>);
  }
  double* TOT = DR + kPanel * kPanel;
  void* args_df[] = {&A, &ld, &M, &nb, &chunk, &tau, &Pp, &DR, &TOT, &Vb, &ldv, &sync};
  void* args_bar[] = {&A, &ld, &M, &nb, &chunk, &tau, &Pp, &DR, &Vb, &ldv, &sync};
  void** args = M >= nb ? args_df : args_bar;
  int maxb = 0;
  RFM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&maxb, fn, 512, 0));
  RFM_CHECK((int64_t)maxb * num_cus(P.device) >= (int64_t)grid.x, RFM_EDEVICE,
            "QR panel: workgroups cannot all be resident");
  RFM_HIP(hipLaunchCooperativeKernel(fn, grid, dim3(512), args, 0, P.stream));
}

void launch_panel(Problem& P, double* A, int64_t ld, int M, int nb, double* tau, double* Pp, double* DR, double* Vb,
                  int64_t ldv) {
  const int ncu = num_cus(P.device);
  int G = std::max(1, std::min(std::min(ncu, 256), (M + 63) / 64));
  int chunk = (M + G - 1) / G;
  const int need = (chunk + 7) / 8;
  ProfScope ps(P.prof, P.stream, "qr_panel", 4.0 * M * (double)nb * nb, 16.0 * M * (double)nb);
  dim3 grid(G);
  if (need <= 8) launch_panel_t<8>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 16) launch_panel_t<16>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 24) launch_panel_t<24>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 32) launch_panel_t<32>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 40) launch_panel_t<40>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else if (need <= 52) launch_panel_t<52>(P, grid, A, ld, M, nb, chunk, tau, Pp, DR, Vb, ldv);
  else throw Error(RFM_EINVAL, "QR panel: too many rows per workgroup (sketch too tall)");
}

}  // namespace

// split-row count for the TN products: enough workgroups to fill the chip,
// at least 256 rows per split, krange a multiple of 32
static void tn_split(int M, int ntile, int ncu, int cap, int* nsplit, int* krange) {
  int ns = std::max(1, std::min(cap, (4 * ncu + ntile - 1) / ntile));
  ns = std::max(1, std::min(ns, M / 256));
  int kr = ((M + ns - 1) / ns + 31) / 32 * 32;
  *krange = kr;
  *nsplit = (M + kr - 1) / kr;
}

// split-row count for the 128 x 128-tile TN products: the workgroups of one launch run in rounds of
// `slots` (the resident count), each split's workgroups taking 1/ns of the rows, so the launch lasts
// about ceil(tiles ns / slots) / ns full-height rounds.  Take the ns <= cap with the fewest (a small
// charge per split for its partials and their reduction breaks near-ties towards fewer splits), at
// least 256 rows per split, krange a multiple of 32.
static void tn_split_rounds(int M, int tiles, int slots, int cap, int* nsplit, int* krange) {
  int best = 1;
  double best_cost = 1e300;
  const int max_ns = std::max(1, std::min(cap, M / 256));
  for (int ns = 1; ns <= max_ns; ++ns) {
    const double rounds = std::ceil((double)tiles * ns / slots) / ns;
    const double cost = rounds + 0.004 * ns;
    if (cost < best_cost) {
      best_cost = cost;
      best = ns;
    }
  }
  const int kr = ((M + best - 1) / best + 31) / 32 * 32;
  *krange = kr;
  *nsplit = (M + kr - 1) / kr;
}

namespace {

// The blocked Householder QR on one column-major matrix A (leading dimension lda): workspace and the
// steps of one 512-column outer panel.  Workspace is sized for matrices of up to Mmax rows and nmax
// columns.
class QrEngine {
 public:
  QrEngine(Problem& P, int64_t Mmax, int64_t nmax) : P(P), ncu(num_cus(P.device)) {
    const size_t vb = (size_t)(Mmax + 1) * kWide;  // V of a 512-column outer panel, leading dimension M rounded up to even
    const size_t tn = (size_t)max_split * std::max<int64_t>(nmax, kWide) * kWide;
    const size_t small = 5 * kPanel * kPanel + 5 * kBig * kBig + 5 * kOuter * kOuter + kWide * kWide;
    const size_t need = vb + small + (size_t)kPanel * ncu * kPanel + 2 * kPanel * kPanel + tn + (size_t)(nmax + 1) * kWide + 256;
    P.d_ws.resize(need);
    Vw = P.d_ws.p;
    T64 = Vw + vb;                     // 4 blocks of 64 x 64
    T128 = T64 + 4 * kPanel * kPanel;  // 2 blocks of 128 x 128
    G128 = T128 + 2 * kBig * kBig;
    X128 = G128 + kBig * kBig;
    Y128 = X128 + kBig * kBig;
    T256 = Y128 + kBig * kBig;         // 2 blocks of 256 x 256: the two halves of an outer panel
    G256 = T256 + 2 * kOuter * kOuter;
    X256 = G256 + kOuter * kOuter;
    Y256 = X256 + kOuter * kOuter;
    T512 = Y256 + kOuter * kOuter;
    G64 = T512 + kWide * kWide;        // summed 64-wide Gram blocks
    Pp = G64 + kPanel * kPanel;
    DR = Pp + (size_t)kPanel * ncu * kPanel;  // panel partials [64][G][64] (G <= ncu)
    part = DR + 2 * kPanel * kPanel;         // panel diagonal rows and column totals
    W2 = part + tn;
    part_cap = tn;
    int32_t zero3[3] = {0, 0, 0};
    RFM_HIP(hipMemcpyAsync(P.d_sync.p, zero3, sizeof(zero3), hipMemcpyHostToDevice, P.stream));
  }

  // Factor the first min(512, ncols) columns of the M x ncols matrix A (its diagonal starting at A[0])
  // and apply the reflectors to the remaining columns; tau[0 .. 511] receives the reflector scalars.
  // The first 256 columns are factored, applied to the second 256 (K = 256), the second 256
  // factored, the two T merged, and the rest updated once with K = 512.
  void outer_step(double* A, int64_t lda, int M, int64_t ncols, double* tau) {
    const int nbw = (int)std::min<int64_t>(kWide, ncols);
    const int nb0 = std::min(kOuter, nbw), nb1 = nbw - nb0;
    const int64_t Mv = (M + 1) & ~1;  // leading dimension of V: even, so that row pairs load as 16 bytes
    factor256(A, lda, M, 0, nb0, Vw, Mv, T256, tau);
    if (nb1 > 0) {
      trailing(Vw, Mv, kOuter, T256, A + (int64_t)kOuter * lda, lda, M, nb1);
      zero_block(Vw, Mv, kOuter, kOuter, kOuter);  // the second half's reflectors start at row 256
      factor256(A, lda, M, kOuter, nb1, Vw + (int64_t)kOuter * Mv + kOuter, Mv, T256 + kOuter * kOuter, tau);
    }
    const int64_t N = ncols - nbw;
    if (N > 0) {
      // nbw = 512 here; G = V_a^T V_b over rows 256..M-1 (V_b is zero above row 256)
      gram_wide(Vw + kOuter, Vw + (int64_t)kOuter * Mv + kOuter, Mv, M - kOuter, kOuter, G256);
      merge_t(G256, T256, T256 + kOuter * kOuter, X256, Y256, kOuter, T512);
      trailing(Vw, Mv, kWide, T512, A + (int64_t)kWide * lda, lda, M, N);
    }
    RFM_HIP(hipGetLastError());
  }

  // resident workgroups of k_gemm_tn128 on the device (queried once)
  int tn128_slots() {
    if (tn_slots == 0) {
      int per_cu = 0;
      RFM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &per_cu, reinterpret_cast<const void*>(&k_gemm_tn128<true>), 256, 0));
      tn_slots = std::max(1, per_cu) * ncu;
    }
    return tn_slots;
  }

  // the singular / time-out flags raised by the panels and by k_extract_r or k_r_signs
  void check_flags() {
    int32_t flags[3];
    RFM_HIP(hipMemcpyAsync(flags, P.d_sync.p, sizeof(flags), hipMemcpyDeviceToHost, P.stream));
    RFM_HIP(hipStreamSynchronize(P.stream));
    RFM_CHECK(flags[kSyncError] == 0, RFM_EDEVICE, "QR panel: a cross-workgroup wait timed out");
    RFM_CHECK(flags[kSyncSingular] == 0, RFM_ESINGULAR, "R has a zero or non-finite diagonal entry");
  }

  void fill(double* p, int64_t cnt, double v = 0.0) {
    if (cnt > 0)
      hipLaunchKernelGGL(k_fill, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, P.stream, p, cnt, v);
  }

 private:
  Problem& P;
  const int ncu;
  int tn_slots = 0;
  static constexpr int max_split = 16;
  double *Vw, *T64, *T128, *G128, *X128, *Y128, *T256, *G256, *X256, *Y256, *T512, *G64, *Pp, *DR, *part, *W2;
  size_t part_cap = 0;  // doubles of split partials

  void zero_block(double* V, int64_t ldv, int c0, int ncols, int nrows) {
    const int64_t cnt = (int64_t)ncols * nrows;
    if (cnt > 0)
      hipLaunchKernelGGL(k_zero_block, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, P.stream, V, ldv, c0, ncols,
                         nrows);
  }
  // merged T of two reflector blocks of width w: [[Ta, -Ta G Tb], [0, Tb]] with G = Va^T Vb
  void merge_t(const double* G, const double* Ta, const double* Tb, double* X, double* Y, int w, double* Tout) {
    const unsigned g1 = (unsigned)((w * w + 255) / 256), g4 = (unsigned)((4 * w * w + 255) / 256);
    hipLaunchKernelGGL(k_sq_gemm, dim3(g1), dim3(256), 0, P.stream, G, Tb, 1.0, w, X);
    hipLaunchKernelGGL(k_sq_gemm, dim3(g1), dim3(256), 0, P.stream, Ta, X, -1.0, w, Y);
    hipLaunchKernelGGL(k_assemble_t, dim3(g4), dim3(256), 0, P.stream, Ta, Tb, Y, w, Tout);
  }
  // split-row Gram V_a^T V_b of two w-wide (128 or 256) column blocks over K rows into G (w x w)
  void gram_wide(const double* Va, const double* Vbk, int64_t ldv, int K, int w, double* G) {
    int nsplit, krange;
    // up to 64 row splits: the Gram is short and wide, and 16 splits leave most CUs idle
    tn_split(K, (w / kBig) * (w / kBig), ncu, 64, &nsplit, &krange);
    krange = (krange + kKC - 1) / kKC * kKC;
    nsplit = (K + krange - 1) / krange;
    RFM_CHECK((size_t)nsplit * w * w <= part_cap, RFM_EINVAL, "QR: Gram partials exceed the workspace");
    RFM_CHECK((int64_t)kBig * ldv * 8 < (int64_t(1) << 32), RFM_EINVAL, "QR: sketch too tall for 32-bit tile offsets");
    hipLaunchKernelGGL((k_gemm_tn128<true, true>), dim3((w / kBig) * (w / kBig) * nsplit), dim3(256), 0, P.stream, Va,
                       ldv, Vbk, ldv, K, w, krange, part, w);
    hipLaunchKernelGGL(k_gsum, dim3((unsigned)((w * w + 255) / 256)), dim3(256), 0, P.stream, part, nsplit, w, G);
  }
  void gram_t(const double* V, int64_t ldv, int K, int nb, const double* tau, double* Tout) {
    int nsplit, krange;
    tn_split(K, 1, ncu, 256, &nsplit, &krange);
    hipLaunchKernelGGL(k_gemm_tn, dim3(1, nsplit), dim3(256), 0, P.stream, V, ldv, V, ldv, K, nb, krange, part);
    hipLaunchKernelGGL(k_gsum64, dim3((unsigned)((nb * kPanel + 255) / 256)), dim3(256), 0, P.stream, part, nsplit,
                       nb, G64);
    hipLaunchKernelGGL(k_build_t, dim3(1), dim3(256), 0, P.stream, G64, 1, nb, tau, Tout);
  }
  // C (M x N at Cp, leading dimension ldc) <- (I - V T^T V^T) C for the K = 256 or 512 reflectors in
  // V (leading dimension Mv): W = V^T C, W2 = -T^T W, C += V W2^T
  void trailing(const double* V, int64_t Mv, int K, const double* T, double* Cp, int64_t ldc, int M, int64_t N) {
    const int ntile = (int)((N + kBig - 1) / kBig);
    const int halves = K / kBig;
    int nsplit, krange;
    tn_split_rounds(M, halves * ntile, tn128_slots(), max_split, &nsplit, &krange);
    krange = (krange + kKC - 1) / kKC * kKC;
    nsplit = (M + krange - 1) / krange;
    {
      ProfScope ps(P.prof, P.stream, "qr_gemm_tn", 2.0 * M * (double)N * K,
                   8.0 * (2.0 * M * N + (double)M * K + (double)nsplit * N * K));
      // 16-byte loads of C need an even leading dimension and an aligned first column
      const bool vec = (ldc % 2 == 0) && (reinterpret_cast<uintptr_t>(Cp) % 16 == 0);
      RFM_CHECK((int64_t)kBig * std::max<int64_t>(Mv, ldc) * 8 < (int64_t(1) << 32), RFM_EINVAL,
                "QR: sketch too tall for 32-bit tile offsets");
      if (vec)
        hipLaunchKernelGGL(k_gemm_tn128<true>, dim3(halves * ntile * nsplit), dim3(256), 0, P.stream, V, Mv, Cp, ldc,
                           M, (int)N, krange, part, K);
      else
        hipLaunchKernelGGL(k_gemm_tn128<false>, dim3(halves * ntile * nsplit), dim3(256), 0, P.stream, V, Mv, Cp, ldc,
                           M, (int)N, krange, part, K);
    }
    const int64_t ldw = (N + 1) & ~(int64_t)1;  // even, so that column pairs load as 16 bytes
    if (K == kWide)
      hipLaunchKernelGGL(k_reduce_wide<kWide>, dim3((unsigned)((N + 7) / 8)), dim3(kWide), 0, P.stream, part, nsplit,
                         (int)N, T, W2, ldw);
    else
      hipLaunchKernelGGL(k_reduce_wide<kOuter>, dim3((unsigned)((N + 7) / 8)), dim3(kOuter), 0, P.stream, part,
                         nsplit, (int)N, T, W2, ldw);
    {
      ProfScope ps(P.prof, P.stream, "qr_gemm_nn", 2.0 * M * (double)N * K,
                   8.0 * (2.0 * M * N + (double)M * K + (double)N * K));
      RFM_CHECK(Mv % 2 == 0 && Mv >= M && K % (2 * kKC) == 0 && reinterpret_cast<uintptr_t>(V) % 16 == 0 &&
                    reinterpret_cast<uintptr_t>(W2) % 16 == 0,
                RFM_EINVAL, "QR: trailing-update operands not laid out for 16-byte loads");
      hipLaunchKernelGGL(k_gemm_nn128, dim3((unsigned)((M + kBig - 1) / kBig * ntile)), dim3(256), 0, P.stream, Cp,
                         ldc, V, Mv, W2, ldw, M, (int)N, K);
    }
  }
  // Factor columns c0 .. c0 + nbh - 1 (nbh <= 256) of the M-row matrix A (diagonal at A[0]) in four
  // 64-column blocks; their reflectors go to Vh (row 0 = row c0 of A, leading dimension Mv) and the T
  // of all of them to Tout.
  void factor256(double* A, int64_t lda, int M, int c0, int nbh, double* Vh, int64_t Mv, double* Tout, double* tau) {
    const int Mh = M - c0;
    const int nsp = (nbh + kPanel - 1) / kPanel;
    // V columns of blocks beyond the last one stay zero
    if (nsp < 4) zero_block(Vh, Mv, nsp * kPanel, (4 - nsp) * kPanel, Mh);
    if (nsp < 4) fill(T64 + (size_t)nsp * kPanel * kPanel, (int64_t)(4 - nsp) * kPanel * kPanel);
    int nbs[4] = {0, 0, 0, 0};
    for (int sp = 0; sp < nsp; ++sp) {
      const int64_t c_sp = c0 + (int64_t)sp * kPanel;
      const int Msp = Mh - sp * kPanel;
      const int nbsp = std::min(kPanel, nbh - sp * kPanel);
      nbs[sp] = nbsp;
      double* Vsp = Vh + (int64_t)sp * kPanel * Mv + sp * kPanel;
      if (sp > 0) zero_block(Vh, Mv, sp * kPanel, kPanel, sp * kPanel);
      launch_panel(P, A + c_sp * lda + c_sp, lda, Msp, nbsp, tau + c_sp, Pp, DR, Vsp, Mv);
      gram_t(Vsp, Mv, Msp, nbsp, tau + c_sp, T64 + (size_t)sp * kPanel * kPanel);
      const int Nr = nbh - (sp + 1) * kPanel;
      if (Nr > 0) {
        // apply this block's reflectors to the rest of the 256 columns
        double* Cr = A + (c_sp + kPanel) * lda + c_sp;
        int nsplit, krange;
        tn_split(Msp, (Nr + 63) / 64, ncu, 256, &nsplit, &krange);
        hipLaunchKernelGGL(k_gemm_tn, dim3((unsigned)((Nr + 63) / 64), nsplit), dim3(256), 0, P.stream, Vsp, Mv, Cr,
                           lda, Msp, Nr, krange, part);
        hipLaunchKernelGGL(k_reduce_w, dim3((unsigned)((Nr + 3) / 4)), dim3(256), 0, P.stream, part, nsplit, Nr,
                           T64 + (size_t)sp * kPanel * kPanel, W2);
        hipLaunchKernelGGL(k_gemm_nn, dim3((unsigned)((Msp + 63) / 64), (unsigned)((Nr + 63) / 64)), dim3(256), 0,
                           P.stream, Cr, lda, Vsp, Mv, W2, Msp, Nr, kPanel);
      }
    }
    // T of the 256 reflectors: pairs of 64-blocks into 128-blocks, then the two 128-blocks
    for (int pr = 0; pr < 2; ++pr) {
      const int a = 2 * pr, b = 2 * pr + 1;
      int nsplit_ab = 1, krange;
      const int Kab = Mh - b * kPanel;
      if (nbs[b] > 0) {
        tn_split(Kab, 1, ncu, 256, &nsplit_ab, &krange);
        hipLaunchKernelGGL(k_gemm_tn, dim3(1, nsplit_ab), dim3(256), 0, P.stream, Vh + (int64_t)a * kPanel * Mv + b * kPanel,
                           Mv, Vh + (int64_t)b * kPanel * Mv + b * kPanel, Mv, Kab, nbs[b], krange, part);
        hipLaunchKernelGGL(k_gsum64, dim3((unsigned)((nbs[b] * kPanel + 255) / 256)), dim3(256), 0, P.stream, part,
                           nsplit_ab, nbs[b], G64);
      }
      hipLaunchKernelGGL(k_combine_t, dim3(1), dim3(256), 0, P.stream, T64 + (size_t)a * kPanel * kPanel,
                         T64 + (size_t)b * kPanel * kPanel, G64, 1, nbs[b], T128 + (size_t)pr * kBig * kBig);
    }
    // G = V01^T V23 over rows 128..Mh-1 (V23 is zero above row 128)
    if (nsp > 2 && Mh > kBig) gram_wide(Vh + kBig, Vh + (int64_t)kBig * Mv + kBig, Mv, Mh - kBig, kBig, G128);
    else fill(G128, (int64_t)kBig * kBig);  // no reflectors past column 128 in this block
    merge_t(G128, T128, T128 + kBig * kBig, X128, Y128, kBig, Tout);
    RFM_HIP(hipGetLastError());
  }
};

}  // namespace

void qr_factor(Problem& P) {
  const int64_t s = P.s, n = P.n;
  RFM_CHECK(s >= n, RFM_EINVAL, "QR: sketch has fewer rows than columns");
  QrEngine E(P, s, n);
  P.d_tau.resize(n);
  double* B = P.d_B.p;
  for (int64_t col0 = 0; col0 < n; col0 += kWide)
    E.outer_step(B + col0 * s + col0, s, (int)(s - col0), n - col0, P.d_tau.p + col0);
  // R to tiled storage
  const int nbt = (int)((n + kTB - 1) / kTB);
  P.d_R.resize((size_t)nbt * (nbt + 1) / 2 * kTB * kTB);
  hipLaunchKernelGGL(k_extract_r, dim3(nbt, nbt), dim3(256), 0, P.stream, B, s, (int)n, P.d_R.p, P.d_sync.p);
  RFM_HIP(hipGetLastError());
  E.check_flags();
  prepare_trsv(P);
}

int64_t qr_stream_rows(const Problem& P, int64_t want) {
  const int64_t s = P.s, n = P.n;
  int64_t b;
  if (want > 0) {
    b = want;
  } else {
    size_t fr = 0, tot = 0;
    RFM_HIP(hipMemGetInfo(&fr, &tot));
    // the sketch rows of one pass and the 512-row top slot in about an eighth of the device memory
    b = (int64_t)((double)tot / 8.0 / (8.0 * (double)n)) - kWide;
  }
  // the panel kernel holds at most 52 rows per thread row of its 256 workgroups (106,496 rows)
  b = std::min<int64_t>(b, 98304);
  b = std::max<int64_t>(kBig, b / kBig * kBig);
  return std::min<int64_t>(b, (s + kBig - 1) / kBig * kBig);
}

double streamed_sketch_qr(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int pieces, int64_t rows_per_pass) {
  const auto t0 = std::chrono::steady_clock::now();
  if (prec != RFM_PREC_F64) {
    launch_cast_panels(P, prec, pieces);
    RFM_HIP(hipStreamSynchronize(P.stream));
  }
  const double t_cast = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  auto rows = [&](int64_t r0, int64_t nr, double* out, int64_t ldo) {
    if (prec == RFM_PREC_F64)
      launch_sketch_rows(P, seed, jac_index, r0, nr, out, ldo);
    else
      launch_sketch_lowp_rows(P, seed, jac_index, prec, r0, nr, out, ldo);
  };
  return t_cast + qr_factor_streamed(P, rows, qr_stream_rows(P, rows_per_pass));
}

bool qr_should_stream(const Problem& P) {
  size_t fr = 0, tot = 0;
  RFM_HIP(hipMemGetInfo(&fr, &tot));
  const int64_t nbt = (P.n + kTB - 1) / kTB;
  const double r_bytes = (double)nbt * (nbt + 1) / 2 * kTB * kTB * 8.0;
  // B, R and the QR's split partials in at most 60% of the device memory
  const double need = 8.0 * (double)P.s * P.n + r_bytes + 8.0 * 16.0 * kWide * (double)std::max<int64_t>(P.n, kWide);
  return need > 0.6 * (double)tot;
}

double qr_factor_streamed(Problem& P, const std::function<void(int64_t, int64_t, double*, int64_t)>& sketch_rows,
                          int64_t rows_per_pass) {
  const int64_t s = P.s, n = P.n;
  RFM_CHECK(s >= n, RFM_EINVAL, "QR: sketch has fewer rows than columns");
  RFM_CHECK(rows_per_pass >= kBig && rows_per_pass % kBig == 0, RFM_EINVAL,
            "streamed QR: rows per pass must be a positive multiple of 128");
  const int64_t b = std::min<int64_t>(rows_per_pass, (s + kBig - 1) / kBig * kBig);
  const int64_t ldy = kWide + b;  // 512-row slot for R's rows above the pass's sketch rows
  RFM_CHECK((double)ldy * n < 9e18 / 8, RFM_EINVAL, "streamed QR: buffer too large");
  P.d_B.resize((size_t)ldy * n);
  double* Y = P.d_B.p;
  QrEngine E(P, ldy, n);
  P.d_tau.resize(std::max<int64_t>(n, kWide));
  const int nbt = (int)((n + kTB - 1) / kTB);
  const size_t rsz = (size_t)nbt * (nbt + 1) / 2 * kTB * kTB;
  P.d_R.resize(rsz);
  E.fill(P.d_R.p, (int64_t)rsz);  // R = 0 before the first pass
  double t_sketch = 0.0;
  for (int64_t r0 = 0; r0 < s; r0 += b) {
    const int64_t nr = std::min<int64_t>(b, s - r0);
    // sketch rows r0 .. r0 + nr - 1 below the slot
    RFM_HIP(hipStreamSynchronize(P.stream));
    const auto t0 = std::chrono::steady_clock::now();
    sketch_rows(r0, nr, Y + kWide, ldy);
    RFM_HIP(hipStreamSynchronize(P.stream));
    t_sketch += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    // [R; B_pass] = Q R': each outer panel factors R's rows col0 .. col0 + 511 stacked on the pass's
    // rows (R is zero below its diagonal, so the reflectors only touch those rows)
    const int M = (int)(kWide + nr);
    for (int64_t col0 = 0; col0 < n; col0 += kWide) {
      const int64_t ncols = n - col0;
      const unsigned g = (unsigned)((ncols * kWide + 255) / 256);
      hipLaunchKernelGGL(k_strip_in, dim3(g), dim3(256), 0, P.stream, P.d_R.p, (int)n, col0, Y, ldy);
      E.outer_step(Y + col0 * ldy, ldy, M, ncols, P.d_tau.p);
      hipLaunchKernelGGL(k_strip_out, dim3(g), dim3(256), 0, P.stream, P.d_R.p, (int)n, col0, Y, ldy);
    }
    RFM_HIP(hipGetLastError());
    if (P.verbose) {
      RFM_HIP(hipStreamSynchronize(P.stream));
      std::fprintf(stderr, "[rfm] streamed QR: sketch rows %lld .. %lld of %lld folded into R\n", (long long)r0,
                   (long long)(r0 + nr), (long long)s);
    }
  }
  // positive diagonal, identity padding, singular check
  hipLaunchKernelGGL(k_r_signs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, P.stream, P.d_R.p, (int)n,
                     P.d_tau.p, P.d_sync.p);
  hipLaunchKernelGGL(k_r_apply_signs, dim3(nbt, nbt), dim3(256), 0, P.stream, P.d_R.p, (int)n, P.d_tau.p);
  RFM_HIP(hipGetLastError());
  E.check_flags();
  prepare_trsv(P);
  return t_sketch;
}

void launch_get_r_cols(Problem& P, int64_t c0, int64_t ncols, double* out) {
  hipLaunchKernelGGL(k_get_r_cols, dim3((unsigned)ncols), dim3(256), 0, P.stream, P.d_R.p, (int)P.n, c0, out);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
