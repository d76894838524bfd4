// Triangular solves with the preconditioner R (Alg. 1 steps 3-5): x = R^{-1} y
// and x = R^{-T} y, R stored as 64 x 64 column-major tiles of its upper triangle.
//
// The solve is a chain over the nb = ceil(n / 64) blocks of x (R x = y from the
// last block up, R^T x = y from the first block down): block i needs every
// block before it in chain order.  One launch of nb + 1 workgroups; each takes
// a ticket from an atomic counter.
//  * Ticket 0 is the solver.  It walks the whole chain and keeps the blocks it
//    solved in LDS, so no step of the chain waits for another workgroup's
//    stores: per block it applies the kLook = 2 tiles next to the diagonal,
//    subtracts the helpers' partial sum for the block, solves the 64 x 64
//    diagonal tile by substitution in LDS and publishes the block.  Its eight wavefronts: 0 solves and publishes, with its row of the
//    diagonal tile in registers (the substitution is the chain's longest part);
//    1-3 and 4-6 are two sets that hold the two off-diagonal tiles and the
//    diagonal tile of even and odd steps in registers, each set loading its next
//    step two steps ahead.  Only the product with the block solved last is left
//    between two substitutions: the product with the block before it and the
//    diagonal tile's copy to LDS are done a step early.  Wavefront 7 fetches the
//    helper partial of the next step (alone, so that its reads do not wait
//    behind tile loads).
//  * Ticket t >= 1 is the helper of block t-th in chain order: it streams the
//    rest of that block's row (R) or column (R^T) of tiles as the solver
//    publishes the blocks they multiply, and publishes the partial sum.  It
//    needs blocks up to kLook + 1 steps behind the one it serves, so the solver
//    finds the partial ready.
// Published data are written and read with device-scope relaxed atomics
// (coherent across the XCDs' L2s), and every published value carries its own
// ready state: a fill kernel sets every slot of the blocks of x and of the
// helpers' partial sums to a signalling-NaN pattern that no result has (a NaN
// result is stored as the canonical quiet NaN) before the launch; a writer
// stores its values and moves on -- no wait for the stores to be acknowledged,
// no flag -- and a reader takes a block once none of its 64 slots holds the
// pattern.  The solver reads the next step's partial a phase before it needs
// it, so one round trip to memory per step is hidden behind the substitution.
// Workgroups only wait for work of smaller tickets (the solver waits for
// helpers of blocks whose dependencies it has already published, and helpers
// start in the order the solver needs them), so the launch always drains; a
// spin limit turns a lost value into an error instead of a hang.
//
// Optional fusion for LSQR: out = yscale-scaled solve minus coef * sub, and a
// per-block partial of ||out||^2.
#include "rfm_internal.h"

namespace rfm {

namespace {

constexpr int kTB = 64;
constexpr int kSpinLimit = 1 << 26;
constexpr int kLook = 2;   // off-diagonal tiles next to the diagonal applied by the solver
constexpr int kBatch = 8;  // helper: upcoming blocks read per round trip
// sync words used here: [8] ticket counter, [9] error flag
enum { kTicket = 8, kTrsvErr = 9 };

__device__ __forceinline__ const double* tile_ptr(const double* Rt, int bi, int bj) {
  return Rt + ((size_t)bj * (bj + 1) / 2 + bi) * kTB * kTB;
}

__device__ __forceinline__ double ld_dev(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_dev(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int ld_flag(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// an empty slot of a published block of x: a signalling-NaN bit pattern no result takes
constexpr uint64_t kEmpty = 0x7FF4F00DDEADBEEFull;
__device__ __forceinline__ double canon(double v) {  // a NaN result becomes the canonical quiet NaN
  return v != v ? __longlong_as_double(0x7FF8000000000000ll) : v;
}
__device__ __forceinline__ bool filled(double v) { return (uint64_t)__double_as_longlong(v) != kEmpty; }

__global__ void __launch_bounds__(256) k_trsv_clear(double* __restrict__ z, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) z[i] = __longlong_as_double((long long)kEmpty);
}

__device__ __forceinline__ double bcast(double v, int k) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, k);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), k);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// mode 0: R x = y   (chain from the last block up)
// mode 1: R^T x = y (chain from the first block down)
template <int MODE>
__global__ void __launch_bounds__(512) k_trsv(const double* __restrict__ Rt, int n, int nbk,
                                              const double* __restrict__ y, double* __restrict__ z,
                                              double* __restrict__ pz, double* __restrict__ out,
                                              const double* __restrict__ sub, const LsqrState* __restrict__ st,
                                              int yscale_sel, int sub_sel, double* __restrict__ partial,
                                              int32_t* __restrict__ sync) {
  if (st && st->done) return;
  __shared__ int tk_sh;
  __shared__ double Dt[2][kTB][kTB + 1];  // solver: diagonal tiles of even and odd steps, [row][col], diagonal zeroed
  __shared__ double dg[2][kTB];           // solver: their diagonals
  __shared__ double xs[kBatch][kTB];    // helper: ready blocks of x
  __shared__ double red[8][kTB];
  __shared__ double xl[kLook][kTB];     // solver: the last kLook solved blocks (by step parity)
  __shared__ double pzs[2][kTB];        // solver: helper partials of this and the next step
  __shared__ double red2[2][kTB];       // solver: product with the block two steps back
  __shared__ int nready_sh;
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  if (tid == 0) {
    const int t = __hip_atomic_fetch_add(&sync[kTicket], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (t == nbk) __hip_atomic_store(&sync[kTicket], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    tk_sh = t;
  }
  __syncthreads();
  const int ticket = tk_sh;
  constexpr int d = MODE == 0 ? 1 : -1;  // step from a block to the one solved just before it
  auto blk = [&](int step) { return MODE == 0 ? nbk - 1 - step : step; };

  if (ticket == 0) {
    // ------------------------------------------------------------------ solver
    double ysc = 1.0, coef = 0.0;
    if (st) {
      ysc = yscale_sel == 1 ? st->inv_alpha : 1.0;
      coef = sub_sel == 1 ? st->beta * st->inv_alpha : 0.0;
    }
    // wavefronts 1-3 (even steps) and 4-6 (odd steps): role 0 the tile next to the diagonal, 1 the
    // one after, 2 the diagonal tile; lane l holds row l of the tile as the solve sees it (R, or R^T
    // in mode 1).  Wavefront 0 keeps row (mode 0) or column (mode 1) `lane` of the current diagonal
    // tile in the same registers.
    const int set = (wv - 1) / 3, role = (wv - 1) % 3;
    const bool tile_wave = wv >= 1 && wv <= 6;
    double tv[kTB];
    auto load_tiles = [&](int step) {
      const int i = blk(step);
      if (role < 2) {
        const int ij = i + (role == 0 ? d : 2 * d);
        const bool has = ij >= 0 && ij < nbk;
        if (MODE == 0) {
          const double* T = tile_ptr(Rt, i, has ? ij : i);
#pragma unroll
          for (int c = 0; c < kTB; ++c) tv[c] = has ? T[c * kTB + lane] : 0.0;
        } else {
          const double* T = tile_ptr(Rt, has ? ij : i, i);
#pragma unroll
          for (int r = 0; r < kTB; ++r) tv[r] = has ? T[lane * kTB + r] : 0.0;
        }
      } else {
        const double* T = tile_ptr(Rt, i, i);
#pragma unroll
        for (int c = 0; c < kTB; ++c) tv[c] = T[c * kTB + lane];
      }
    };
    // wavefront 7: the helper partial of `step`, a value that is its own ready state; pv holds the
    // first read (issued a phase earlier), re-read until all 64 slots are filled
    auto finish_partial = [&](int step, double pv) {
      const double* src = &pz[(size_t)blk(step) * kTB + lane];
      int spins = 0;
      while (__ballot(filled(pv)) != ~0ull) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 1023) == 0 && ld_flag(&sync[kTrsvErr]) != 0) break;
        if (spins > kSpinLimit) {
          __hip_atomic_store(&sync[kTrsvErr], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
        pv = ld_dev(src);
      }
      pzs[step & 1][lane] = pv;
    };
    double pnext = 0.0;  // wavefront 7: the next step's partial, in flight
    // tile (registers) times a block of x (LDS, read by every lane): the block is read 16 values
    // at a time into registers of their own so that the reads overlap
    auto tile_times = [&](const double* xv) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
      for (int kb = 0; kb < kTB; kb += 16) {
        double xr[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) xr[q] = xv[kb + q];
#pragma unroll
        for (int q = 0; q < 16; q += 4) {
          a0 += tv[kb + q] * xr[q];
          a1 += tv[kb + q + 1] * xr[q + 1];
          a2 += tv[kb + q + 2] * xr[q + 2];
          a3 += tv[kb + q + 3] * xr[q + 3];
        }
      }
      return (a0 + a1) + (a2 + a3);
    };
    auto two_back = [&](int step) {  // role 1 of the set of `step`: its tile times the block of step - 2
      red2[step & 1][lane] = tile_times(xl[step & 1]);
    };
    auto diag_to_lds = [&](int step) {  // role 2 of the set of `step`: tile without its diagonal, and the diagonal
      double d = 0.0;
#pragma unroll
      for (int c = 0; c < kTB; ++c) {
        Dt[step & 1][lane][c] = c == lane ? 0.0 : tv[c];
        d = c == lane ? tv[c] : d;
      }
      dg[step & 1][lane] = d;
    };
    // wavefront 0: y (and sub) of the next kYAhead blocks in a register queue, each read kYAhead steps
    // before its block is solved (the helpers keep the memory system busy, so one step is not always
    // enough for a read to return)
    constexpr int kYAhead = 4;
    double yq[kYAhead], sq[kYAhead];
    auto read_y = [&](int step, double& yv, double& sv) {
      const int row = step < nbk ? blk(step) * kTB + lane : n;
      yv = row < n ? y[row] : 0.0;
      sv = (sub && row < n) ? sub[row] : 0.0;
    };
    // wavefront 0: the row (mode 0) or column (mode 1) `lane` of a step's diagonal tile from LDS into
    // registers, divided by its diagonal entry, the entry itself dropped: each unknown is then final
    // when its turn comes, and one FMA per step updates every lane (lanes already solved, and the
    // pivot lane, multiply a zero)
    double rd = 0.0;
    auto prepare_row = [&](int step) {
      const int b = step & 1;
#pragma unroll
      for (int k = 0; k < kTB; ++k) tv[k] = MODE == 0 ? Dt[b][lane][k] : Dt[b][k][lane];
      rd = 1.0 / dg[b][lane];
#pragma unroll
      for (int k = 0; k < kTB; ++k) tv[k] *= rd;
    };
    if (wv == 0) {
      xl[0][lane] = 0.0;
      xl[1][lane] = 0.0;
#pragma unroll
      for (int q = 0; q < kYAhead; ++q) read_y(q, yq[q], sq[q]);
    } else if (tile_wave) {
      if (set < nbk) load_tiles(set);
    } else {
      finish_partial(0, ld_dev(&pz[(size_t)blk(0) * kTB + lane]));
    }
    __syncthreads();
    // step 0 has no earlier blocks: only its diagonal tile; the tiles of the set's next step (2) are
    // loaded as soon as the registers are free
    if (tile_wave && set == 0 && role == 1) {
      red2[0][lane] = 0.0;
      if (2 < nbk) load_tiles(2);
    }
    if (tile_wave && set == 0 && role == 2) {
      diag_to_lds(0);
      if (2 < nbk) load_tiles(2);
    }
    __syncthreads();
    if (wv == 0) prepare_row(0);
    // Every tile is loaded as soon as its wavefront has used the previous one, two steps before it is
    // needed: the helpers keep the memory system busy, and one step is not always enough for a load
    // to return.  Phase 1: the product with the block solved last (role 0 of this step's set), the
    // next step's diagonal tile to LDS (role 2 of the other set), the next partial's first read.
    // Phase 2: the substitution and publication of this step's block, then the next step's row of the
    // diagonal tile into registers (wavefront 0); the next step's product with the block of this
    // step's predecessor (role 1 of the other set); the next partial completed (wavefront 7).
    for (int step = 0; step < nbk; ++step) {
      const int i = blk(step);
      const int cur = step & 1;
      const bool in_set = tile_wave && set == cur;      // tiles of this step
      const bool in_next = tile_wave && set != cur;     // tiles of the next step
      if (in_set && role == 0) {
        // the tile next to the diagonal times the block solved last
        red[1][lane] = tile_times(xl[(step + 1) & 1]);
        if (step + 2 < nbk) load_tiles(step + 2);
      } else if (in_next && role == 2 && step + 1 < nbk) {
        diag_to_lds(step + 1);
        if (step + 3 < nbk) load_tiles(step + 3);
      } else if (wv == 7 && step + 1 < nbk) {
        pnext = ld_dev(&pz[(size_t)blk(step + 1) * kTB + lane]);  // completed in the second phase
      }
      __syncthreads();
      if (wv == 0) {
        const double yv = yq[0], sv = sq[0];
        double r = (yv * ysc - pzs[cur][lane] - (red[1][lane] + red2[cur][lane])) * rd;
        if (MODE == 0) {
#pragma unroll
          for (int k = kTB - 1; k >= 0; --k) r = fma(-tv[k], bcast(r, k), r);
        } else {
#pragma unroll
          for (int k = 0; k < kTB; ++k) r = fma(-tv[k], bcast(r, k), r);
        }
        xl[cur][lane] = r;
        const int row = i * kTB + lane;
        st_dev(&z[row], canon(r));  // padded length: nbk * 64; the value is its own ready state
        const double o = r - coef * sv;
        if (row < n) out[row] = o;
        if (partial) {
          double q = row < n ? o * o : 0.0;
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
          if (lane == 0) partial[i] = q;
        }
#pragma unroll
        for (int q = 0; q + 1 < kYAhead; ++q) {
          yq[q] = yq[q + 1];
          sq[q] = sq[q + 1];
        }
        read_y(step + kYAhead, yq[kYAhead - 1], sq[kYAhead - 1]);
        if (step + 1 < nbk) prepare_row(step + 1);
      } else if (in_next && role == 1 && step + 1 < nbk) {
        // next step: its tile two blocks from the diagonal times the block of step - 1
        two_back(step + 1);
        if (step + 3 < nbk) load_tiles(step + 3);
      } else if (wv == 7) {
        if (step + 1 < nbk) finish_partial(step + 1, pnext);
      }
      __syncthreads();
    }
    return;
  }

  // -------------------------------------------------------------------- helper
  // block i; its tiles against blocks j with |j - i| > kLook, in chain order
  const int i = blk(ticket - 1);
  const int jstop = i + (kLook + 1) * d;  // last block in chain order this helper needs
  double acc = 0.0;            // MODE 0: row lane of the block, columns wv*8 .. +7
  double accT[8];              // MODE 1: columns wv*8 .. +7, rows lane
#pragma unroll
  for (int q = 0; q < 8; ++q) accT[q] = 0.0;
  // this thread's 8 values of the tile that multiplies block jb: R(i, jb) columns wv*8 .. +7 at row
  // lane (mode 0), R(jb, i) rows wv*8 .. +7 at column lane (mode 1, the transposed tile's rows)
  auto load_tile = [&](int jb, double* t) {
    const double* T = MODE == 0 ? tile_ptr(Rt, i, jb) : tile_ptr(Rt, jb, i);
#pragma unroll
    for (int q = 0; q < 8; ++q) t[q] = T[(wv * 8 + q) * kTB + lane];
  };
  auto in_range = [&](int jb) { return MODE == 0 ? jb >= jstop : jb <= jstop; };
  // Blocks of x become ready in chain order.  Per round, wavefront 0 reads the
  // next kBatch upcoming blocks in one round trip and stages every ready one in
  // LDS; all eight wavefronts then multiply them.  The tile of the next block
  // in chain order is always in flight into registers while this one is used,
  // so a block that arrives meets its tile already loaded.
  int j = MODE == 0 ? nbk - 1 : 0;
  double tc[8];
  if (in_range(j)) load_tile(j, tc);
  while (in_range(j)) {
    if (wv == 0) {
      const int cnt = min(kBatch, MODE == 0 ? j - jstop + 1 : jstop - j + 1);
      int ready = 0;
      int spins = 0;
      double xv[kBatch];
      while (true) {
        // one round trip reads the next cnt blocks; a block is ready once all 64 of its slots are filled
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
          xv[b] = b < cnt ? ld_dev(&z[(size_t)(j - d * b) * kTB + lane]) : __longlong_as_double((long long)kEmpty);
        ready = 0;
#pragma unroll
        for (int b = 0; b < kBatch; ++b)
          if (ready == b && __ballot(filled(xv[b])) == ~0ull) ready = b + 1;  // leading run in chain order
        if (ready > 0) break;
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 1023) == 0 && ld_flag(&sync[kTrsvErr]) != 0) {
          ready = cnt;
          break;
        }
        if (spins > kSpinLimit) {
          __hip_atomic_store(&sync[kTrsvErr], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ready = cnt;
          break;
        }
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) xs[b][lane] = b < ready ? xv[b] : 0.0;
      if (lane == 0) nready_sh = ready;
    }
    __syncthreads();
    const int ready = nready_sh;
    for (int b = 0; b < ready; ++b) {
      const int jb = j - d * b;
      double tn[8];
      const bool more = in_range(jb - d);
      if (more) load_tile(jb - d, tn);  // the next block's tile, in flight during this product
      if (MODE == 0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) acc += tc[q] * xs[b][wv * 8 + q];
      } else {
        const double zl = xs[b][lane];
#pragma unroll
        for (int q = 0; q < 8; ++q) accT[q] += tc[q] * zl;
      }
      if (more) {
#pragma unroll
        for (int q = 0; q < 8; ++q) tc[q] = tn[q];
      }
    }
    __syncthreads();
    j -= d * ready;
  }
  // combine: red[wv][row] (mode 0) or red[0][column] (mode 1)
  if (MODE == 0) {
    red[wv][lane] = acc;
  } else {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double v = accT[q];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == q) red[0][wv * 8 + q] = v;
    }
  }
  __syncthreads();
  if (wv == 0) {
    double v = red[0][lane];
    if (MODE == 0)
      v = ((red[0][lane] + red[1][lane]) + (red[2][lane] + red[3][lane])) +
          ((red[4][lane] + red[5][lane]) + (red[6][lane] + red[7][lane]));
    st_dev(&pz[(size_t)i * kTB + lane], canon(v));  // the value is its own ready state
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
  RFM_CHECK((int64_t)kTrsvErr < (int64_t)P.d_sync.n, RFM_EINVAL, "triangular solve: no sync words");
  P.d_trsv.resize((size_t)2 * nbk * kTB);
  double* z = P.d_trsv.p;                     // published blocks of x, nbk * 64
  double* pz = P.d_trsv.p + (size_t)nbk * kTB;  // helper partials, nbk * 64
  const double nn = (double)P.n;
  const int64_t nz = 2 * (int64_t)nbk * kTB;  // z and pz are contiguous
  hipLaunchKernelGGL(k_trsv_clear, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, P.stream, z, nz);
  ProfScope ps(P.prof, P.stream, "trsv", nn * nn, 8.0 * (nn * (nn + 1) / 2 + 3 * nn));
  if (transpose)
    hipLaunchKernelGGL(k_trsv<1>, dim3(nbk + 1), dim3(512), 0, P.stream, P.d_R.p, (int)P.n, nbk, y, z, pz, x,
                       sub_vec, st, yscale_sel, sub_sel, red_partials, P.d_sync.p);
  else
    hipLaunchKernelGGL(k_trsv<0>, dim3(nbk + 1), dim3(512), 0, P.stream, P.d_R.p, (int)P.n, nbk, y, z, pz, x,
                       sub_vec, st, yscale_sel, sub_sel, red_partials, P.d_sync.p);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
