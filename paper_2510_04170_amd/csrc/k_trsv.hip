// Triangular solves with the preconditioner R (Alg. 1 steps 3-5): x = R^{-1} y
// and x = R^{-T} y, R stored as 64 x 64 column-major tiles of its upper triangle.
//
// One launch of nb = ceil(n / 64) workgroups.  A workgroup takes a ticket from
// an atomic counter and solves row block i = nb-1-ticket (R x = y) or
// i = ticket (R^T x = y).  It streams its off-diagonal tiles as soon as the
// block of x they multiply is published, then solves the 64 x 64 diagonal
// block by substitution in LDS and publishes its own block (data, release
// fence, per-block flag = epoch).  A workgroup only waits for blocks held by
// workgroups with smaller tickets, which are already running, so the launch
// always drains; a spin limit turns a lost flag into an error instead of a hang.
//
// Optional fusion for LSQR: out = yscale-scaled solve minus coef * sub, and a
// per-block partial of ||out||^2.
#include "rfm_internal.h"

namespace rfm {

namespace {

constexpr int kTB = 64;
constexpr int kSpinLimit = 1 << 26;
// sync words used here: [8] ticket counter, [9] error flag, [16 ...] block flags
enum { kTicket = 8, kTrsvErr = 9, kFlags = 16 };
constexpr int kBatch = 8;  // flags polled per round trip

__device__ __forceinline__ const double* tile_ptr(const double* Rt, int bi, int bj) {
  return Rt + ((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB;
}

// Cross-workgroup handoff without cache maintenance: the published block of x
// and its flag are written and read with device-scope relaxed atomics (sc1,
// coherent across the XCDs' L2s); the writer waits for its data stores to be
// acknowledged before it stores the flag.
__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void stores_done() {
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
  __builtin_amdgcn_s_waitcnt(0);
  __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
__device__ __forceinline__ double bcast(double v, int k) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), k);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// mode 0: R x = y   (back substitution over row blocks)
// mode 1: R^T x = y (forward substitution over column blocks)
template <int MODE>
__global__ void __launch_bounds__(256) k_trsv(const double* __restrict__ Rt, int n, int nbk,
                                              const double* __restrict__ y, double* __restrict__ z,
                                              double* __restrict__ out, const double* __restrict__ sub,
                                              const LsqrState* __restrict__ st, int yscale_sel, int sub_sel,
                                              double* __restrict__ partial, int32_t* __restrict__ sync,
                                              int32_t epoch) {
  if (st && st->done) return;
  __shared__ int tk_sh;
  __shared__ double Dt[kTB][kTB + 1];
  __shared__ double rhs[kTB];
  __shared__ double rdiag[kTB];
  __shared__ double xs[kBatch][kTB];
  __shared__ int nready_sh;
  __shared__ double red[4][kTB];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  if (tid == 0) {
    const int t = __hip_atomic_fetch_add(&sync[kTicket], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t == nbk - 1) __hip_atomic_store(&sync[kTicket], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tk_sh = t;
  }
  __syncthreads();
  const int ticket = tk_sh;
  const int i = MODE == 0 ? nbk - 1 - ticket : ticket;
  double ysc = 1.0, coef = 0.0;
  if (st) {
    ysc = yscale_sel == 1 ? st->inv_alpha : 1.0;
    coef = sub_sel == 1 ? st->beta * st->inv_alpha : 0.0;
  }

  // diagonal tile to LDS first: it does not depend on any other block
  {
    const double* T = tile_ptr(Rt, i, i);
    for (int e = tid; e < kTB * kTB; e += 256) Dt[e % kTB][e / kTB] = T[e];
  }
  __syncthreads();
  if (tid < kTB) rdiag[tid] = 1.0 / Dt[tid][tid];

  // off-diagonal contributions
  double acc = 0.0;            // MODE 0: row lane of the block, columns quarter wv
  double accT[16];             // MODE 1: columns wv*16 .. +15, rows lane
#pragma unroll
  for (int q = 0; q < 16; ++q) accT[q] = 0.0;
  // the tile multiplying the block this one waits for last sits on the critical
  // path: load this thread's 16 values of it before any waiting
  double tl[16];
  {
    const int jl = MODE == 0 ? i + 1 : i - 1;
    const bool has = MODE == 0 ? jl < nbk : jl >= 0;
    const double* T = has ? (MODE == 0 ? tile_ptr(Rt, i, jl) : tile_ptr(Rt, jl, i)) : nullptr;
#pragma unroll
    for (int q = 0; q < 16; ++q) tl[q] = has ? T[(wv * 16 + q) * kTB + lane] : 0.0;
  }
  // Blocks of x become ready in chain order.  Per step, wavefront 0 polls the
  // flags of up to kBatch upcoming blocks in one round trip, loads every ready
  // block once into LDS, and all four wavefronts then stream those tiles.
  if (MODE == 0) {
    int j = nbk - 1;
    while (j > i) {
      if (wv == 0) {
        const int cnt = min(kBatch, j - i);
        int ready = 0;
        int spins = 0;
        while (true) {
          int ok = 0;  // lanes past cnt count as not ready, so ~bal has a set bit at or below cnt
          if (lane < cnt) ok = __hip_atomic_load(&sync[kFlags + j - lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
          const unsigned long long bal = __ballot(ok);
          ready = __builtin_ctzll(~bal);  // leading run of ready blocks j, j-1, ...
          if (ready > cnt) ready = cnt;
          if (ready > 0) break;
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 1023) == 0 && __hip_atomic_load(&sync[kTrsvErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ready = cnt;
            break;
          }
          if (spins > kSpinLimit) {
            __hip_atomic_store(&sync[kTrsvErr], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ready = cnt;
            break;
          }
        }
        double xv[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) xv[b] = b < ready ? ld_dev(&z[(size_t)(j - b) * kTB + lane]) : 0.0;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) xs[b][lane] = xv[b];
        if (lane == 0) nready_sh = ready;
      }
      __syncthreads();
      const int ready = nready_sh;
      for (int b = 0; b < ready; ++b) {
        if (j - b == i + 1) {
#pragma unroll
          for (int q = 0; q < 16; ++q) acc += tl[q] * xs[b][wv * 16 + q];
        } else {
          const double* T = tile_ptr(Rt, i, j - b);
#pragma unroll
          for (int c = wv * 16; c < wv * 16 + 16; ++c) acc += T[c * kTB + lane] * xs[b][c];
        }
      }
      __syncthreads();
      j -= ready;
    }
  } else {
    int j = 0;
    while (j < i) {
      if (wv == 0) {
        const int cnt = min(kBatch, i - j);
        int ready = 0;
        int spins = 0;
        while (true) {
          int ok = 0;  // lanes past cnt count as not ready, so ~bal has a set bit at or below cnt
          if (lane < cnt) ok = __hip_atomic_load(&sync[kFlags + j + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == epoch;
          const unsigned long long bal = __ballot(ok);
          ready = __builtin_ctzll(~bal);
          if (ready > cnt) ready = cnt;
          if (ready > 0) break;
          __builtin_amdgcn_s_sleep(1);
          if ((++spins & 1023) == 0 && __hip_atomic_load(&sync[kTrsvErr], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            ready = cnt;
            break;
          }
          if (spins > kSpinLimit) {
            __hip_atomic_store(&sync[kTrsvErr], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            ready = cnt;
            break;
          }
        }
        double xv[kBatch];
#pragma unroll
        for (int b = 0; b < kBatch; ++b) xv[b] = b < ready ? ld_dev(&z[(size_t)(j + b) * kTB + lane]) : 0.0;
#pragma unroll
        for (int b = 0; b < kBatch; ++b) xs[b][lane] = xv[b];
        if (lane == 0) nready_sh = ready;
      }
      __syncthreads();
      const int ready = nready_sh;
      for (int b = 0; b < ready; ++b) {
        const double zl = xs[b][lane];
        if (j + b == i - 1) {
#pragma unroll
          for (int q = 0; q < 16; ++q) accT[q] += tl[q] * zl;
        } else {
          const double* T = tile_ptr(Rt, j + b, i);
#pragma unroll
          for (int q = 0; q < 16; ++q) accT[q] += T[(wv * 16 + q) * kTB + lane] * zl;
        }
      }
      __syncthreads();
      j += ready;
    }
  }
  // combine: red[wv][row]
  if (MODE == 0) {
    red[wv][lane] = acc;
  } else {
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      double v = accT[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == q) red[0][wv * 16 + q] = v;
    }
  }
  __syncthreads();
  if (tid < kTB) {
    const int row = i * kTB + tid;
    const double yv = row < n ? y[row] * ysc : 0.0;
    const double s = MODE == 0 ? (red[0][tid] + red[1][tid]) + (red[2][tid] + red[3][tid]) : red[0][tid];
    rhs[tid] = yv - s;
  }
  __syncthreads();
  // substitution inside the diagonal tile, one wavefront
  if (wv == 0) {
    double r = rhs[lane];
    if (MODE == 0) {
#pragma unroll
      for (int k = kTB - 1; k >= 0; --k) {
        const double xk = bcast(r, k) * rdiag[k];
        if (lane == k) r = xk;
        else if (lane < k) r -= Dt[lane][k] * xk;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kTB; ++k) {
        const double xk = bcast(r, k) * rdiag[k];
        if (lane == k) r = xk;
        else if (lane > k) r -= Dt[k][lane] * xk;
      }
    }
    const int row = i * kTB + lane;
    st_dev(&z[row], r);  // padded length: nbk * 64
    double o = r;
    if (sub && row < n) o = r - coef * sub[row];
    if (row < n) out[row] = o;
    if (partial) {
      double q = row < n ? o * o : 0.0;
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
      if (lane == 0) partial[i] = q;
    }
  }
  if (wv == 0) {
    stores_done();
    if (lane == 0) __hip_atomic_store(&sync[kFlags + i], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

}  // namespace

int trsv_block() { return kTB; }

// report (and clear) a dependency wait that hit its spin limit in an earlier solve
void check_trsv_error(Problem& P) {
  int32_t err = 0;
  RFM_HIP(hipMemcpyAsync(&err, P.d_sync.p + kTrsvErr, sizeof(err), hipMemcpyDeviceToHost, P.stream));
  RFM_HIP(hipStreamSynchronize(P.stream));
  if (err) {
    const int32_t zero = 0;
    RFM_HIP(hipMemcpy(P.d_sync.p + kTrsvErr, &zero, sizeof(zero), hipMemcpyHostToDevice));
    throw Error(RFM_EDEVICE, "triangular solve: dependency wait timed out");
  }
}

// x = R^{-1} (y * yscale) or R^{-T} (y * yscale); with st != null the scale and the
// subtraction coefficient come from the LSQR state.  sub_vec may alias x.
void launch_trsv(Problem& P, const double* y, double* x, bool transpose, const double* sub_vec,
                 const LsqrState* st, int yscale_sel, int sub_sel, double* red_partials) {
  const int nbk = (int)((P.n + kTB - 1) / kTB);
  RFM_CHECK(kFlags + nbk <= (int)P.d_sync.n, RFM_EINVAL, "triangular solve: too many blocks");
  double* z = P.d_vec.p + 4 * std::max(P.m, P.n);  // padded solution (nbk * 64 <= n + 63)
  RFM_CHECK(4 * std::max(P.m, P.n) + (int64_t)nbk * kTB <= (int64_t)P.d_vec.n, RFM_EINVAL, "scratch too small");
  const double nn = (double)P.n;
  ProfScope ps(P.prof, P.stream, "trsv", nn * nn, 8.0 * (nn * (nn + 1) / 2 + 3 * nn));
  int32_t epoch = (int32_t)(++P.trsv_epoch & 0x7fffffff);
  if (epoch == 0) epoch = (int32_t)(++P.trsv_epoch & 0x7fffffff);
  if (transpose)
    hipLaunchKernelGGL(k_trsv<1>, dim3(nbk), dim3(256), 0, P.stream, P.d_R.p, (int)P.n, nbk, y, z, x, sub_vec, st,
                       yscale_sel, sub_sel, red_partials, P.d_sync.p, epoch);
  else
    hipLaunchKernelGGL(k_trsv<0>, dim3(nbk), dim3(256), 0, P.stream, P.d_R.p, (int)P.n, nbk, y, z, x, sub_vec, st,
                       yscale_sel, sub_sel, red_partials, P.d_sync.p, epoch);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
