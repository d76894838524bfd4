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
//    diagonal tile by substitution and publishes the block.  It reads those
//    three tiles from a copy made once per R (k_trsv_tiles): the diagonal tile
//    with each row already divided by its pivot, each tile laid out so that a
//    lane's 64 values arrive in 16-byte loads.  Its eight wavefronts: 1-3 and
//    4-6 are two sets that hold the two off-diagonal tiles and the diagonal
//    tile of even and odd steps in registers; the diagonal tile's wavefront
//    substitutes and publishes its set's blocks.  Only the product with the
//    block solved last is left between two substitutions: the product with the
//    block before it is done a step early.  Wavefront 7 fetches the helper
//    partial of the next step (alone, so that its reads do not wait behind tile
//    loads); wavefront 0 reads y (and sub) ahead and writes the output.
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
constexpr int kTT = kTB * kTB;
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
__global__ void __launch_bounds__(512) k_trsv(const double* __restrict__ Rt, const double* __restrict__ tiles,
                                              int n, int nbk,
                                              const double* __restrict__ y, double* __restrict__ z,
                                              double* __restrict__ pz, double* __restrict__ out,
                                              const double* __restrict__ sub, const LsqrState* __restrict__ st,
                                              int yscale_sel, int sub_sel, double* __restrict__ partial,
                                              int32_t* __restrict__ sync) {
  if (st && st->done) return;
  __shared__ int tk_sh;
  __shared__ double xs[kBatch][kTB];    // helper: ready blocks of x
  __shared__ double red[8][kTB];
  __shared__ double xl[kLook][kTB];     // solver: the last kLook solved blocks (by step parity)
  __shared__ double pzs[2][kTB];        // solver: helper partials of this and the next step
  __shared__ double red2[2][kTB];       // solver: product with the block two steps back
  __shared__ double ysl[2][kTB];        // solver: y of this step's and the next step's block
  __shared__ double ssl[2][kTB];        // solver: sub of the same blocks
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
    // one after, 2 the diagonal tile, each from the solver's copy (zero where the tile would lie past
    // R's edge); lane l holds row l of the tile as the solve sees it (R, or R^T in mode 1).  The
    // diagonal tile's row comes divided by its pivot, the pivot itself dropped: each unknown is then
    // final when its turn comes, and one FMA per step updates every lane (lanes already solved, and
    // the pivot lane, multiply a zero).  Role 2 substitutes and publishes its set's blocks.
    const int set = (wv - 1) / 3, role = (wv - 1) % 3;
    const bool tile_wave = wv >= 1 && wv <= 6;
    const double* Tm = tiles + (size_t)MODE * nbk * 3 * kTT;  // [block][role 2, 0, 1][64 x 64]
    const double* rdv = tiles + (size_t)2 * nbk * 3 * kTT;   // [block][64]: 1 / pivot
    double tv[kTB];
    double rd = 0.0;  // role 2: 1 / pivot of row `lane`
    auto load_tiles = [&](int step) {
      const int i = blk(step);
      // element k of lane l at (k / 2) * 128 + 2 l + k % 2: 16-byte loads, 1 KB per wavefront each
      const double* T = Tm + ((size_t)i * 3 + (role == 2 ? 0 : role + 1)) * kTT + 2 * lane;
#pragma unroll
      for (int k = 0; k < kTB; k += 2) {
        const double2 v = *reinterpret_cast<const double2*>(T + k * kTB);
        tv[k] = v.x;
        tv[k + 1] = v.y;
      }
      if (role == 2) rd = rdv[(size_t)i * kTB + lane];
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
    // wavefront 0: y (and sub) of each block read two steps before its solve and put in LDS a step
    // before it, for the substituting wavefront (y) and for the block's output (sub), which it writes
    // (with its share of ||out||^2) a step after the solve.  The values in flight stay in the same
    // two registers from one step to the next: a queue shifted through registers would make every
    // wavefront wait at the end of each step for all of its own loads in flight, the tile loads too.
    double yn = 0.0, sn = 0.0;
    auto read_y = [&](int step, double& yv, double& sv) {
      const int row = step < nbk ? blk(step) * kTB + lane : n;
      yv = row < n ? y[row] : 0.0;
      sv = (sub && row < n) ? sub[row] : 0.0;
    };
    auto emit = [&](int step, double r, double sv) {
      const int i = blk(step);
      const int row = i * kTB + lane;
      const double o = r - coef * sv;
      if (row < n) out[row] = o;
      if (partial) {
        double q = row < n ? o * o : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) q += __shfl_xor(q, off, 64);
        if (lane == 0) partial[i] = q;
      }
    };
    // prologue: each set's first tiles (the set of step 0 has no tile two blocks back: that product is
    // zero, and its wavefront loads step 2's tile at once)
    if (wv == 0) {
      xl[0][lane] = 0.0;
      xl[1][lane] = 0.0;
      read_y(0, yn, sn);
      ysl[0][lane] = yn;
      ssl[0][lane] = sn;
      read_y(1, yn, sn);
    } else if (tile_wave) {
      if (set == 0 && role == 1) {
        red2[0][lane] = 0.0;
        if (2 < nbk) load_tiles(2);
      } else if (set < nbk) {
        load_tiles(set);
      }
    } else {
      finish_partial(0, ld_dev(&pz[(size_t)blk(0) * kTB + lane]));
    }
    __syncthreads();
    // Each tile is loaded as soon as its wavefront has used the previous one.  Phase 1: the product
    // with the block solved last (role 0 of this step's set), the other set's diagonal tile for the
    // next step (its role 2), the next partial's first read, the last block's output and the next
    // step's y and sub (wavefront 0).  Phase 2: the substitution and publication of this step's block
    // (role 2 of its set); the next step's product with the block of this step's predecessor (role 1
    // of the other set); the next partial completed (wavefront 7).
    for (int step = 0; step < nbk; ++step) {
      const int i = blk(step);
      const int cur = step & 1;
      const bool in_set = tile_wave && set == cur;      // tiles of this step
      const bool in_next = tile_wave && set != cur;     // tiles of the next step
      if (in_set && role == 0) {
        // the tile next to the diagonal times the block solved last
        red[1][lane] = tile_times(xl[(step + 1) & 1]);
        if (step + 2 < nbk) load_tiles(step + 2);
      } else if (in_next && role == 2) {
        if (step >= 1 && step + 1 < nbk) load_tiles(step + 1);
      } else if (wv == 7) {
        if (step + 1 < nbk) pnext = ld_dev(&pz[(size_t)blk(step + 1) * kTB + lane]);  // completed in phase 2
      } else if (wv == 0) {
        if (step >= 1) emit(step - 1, xl[(step + 1) & 1][lane], ssl[(step + 1) & 1][lane]);
        ysl[(step + 1) & 1][lane] = yn;  // y and sub of the next step (past the last block: zeros)
        ssl[(step + 1) & 1][lane] = sn;
        read_y(step + 2, yn, sn);
      }
      __syncthreads();
      if (in_set && role == 2) {
        double r = (ysl[cur][lane] * ysc - pzs[cur][lane] - (red[1][lane] + red2[cur][lane])) * rd;
        if (MODE == 0) {
#pragma unroll
          for (int k = kTB - 1; k >= 0; --k) r = fma(-tv[k], bcast(r, k), r);
        } else {
#pragma unroll
          for (int k = 0; k < kTB; ++k) r = fma(-tv[k], bcast(r, k), r);
        }
        xl[cur][lane] = r;
        st_dev(&z[(size_t)i * kTB + lane], canon(r));  // padded length: nbk * 64; the value is its own ready state
      } else if (in_next && role == 1 && step + 1 < nbk) {
        // next step: its tile two blocks from the diagonal times the block of step - 1
        red2[(step + 1) & 1][lane] = tile_times(xl[(step + 1) & 1]);
        if (step + 3 < nbk) load_tiles(step + 3);
      } else if (wv == 7) {
        if (step + 1 < nbk) finish_partial(step + 1, pnext);
      }
      __syncthreads();
    }
    if (wv == 0) emit(nbk - 1, xl[(nbk - 1) & 1][lane], ssl[(nbk - 1) & 1][lane]);
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

// The solver's copies of the tiles on and next to the diagonal, one workgroup per block i and mode:
// the diagonal tile with each row (mode 0; column, mode 1) divided by its pivot and the pivot dropped,
// then the tiles one and two blocks from the diagonal on the side solved first (zero past R's edge),
// each with lane l's 64 values (row l of the tile as the solve sees it) in 16-byte pairs, pair p of
// lane l at p * 128 + 2 l; after both modes, 1 / pivot of the block's 64 rows.
__global__ void __launch_bounds__(256) k_trsv_tiles(const double* __restrict__ Rt, int nbk, double* __restrict__ tiles) {
  const int i = blockIdx.x, mode = blockIdx.y;
  __shared__ double A[kTB][kTB + 1];  // [row][column] of the source tile
  __shared__ double rds[kTB];
  double* dst = tiles + ((size_t)mode * nbk + i) * 3 * kTT;
  for (int slot = 0; slot < 3; ++slot) {
    const int j = slot == 0 ? i : (mode == 0 ? i + slot : i - slot);
    const bool has = j >= 0 && j < nbk;
    const int jj = has ? j : i;  // an in-bounds stand-in for a tile past the edge, read as zero
    const double* T = mode == 0 ? tile_ptr(Rt, i, jj) : tile_ptr(Rt, jj, i);
    __syncthreads();
    for (int e = threadIdx.x; e < kTT; e += 256) A[e % kTB][e / kTB] = has ? T[e] : 0.0;
    __syncthreads();
    if (slot == 0 && threadIdx.x < kTB) rds[threadIdx.x] = 1.0 / A[threadIdx.x][threadIdx.x];
    __syncthreads();
    for (int o = threadIdx.x; o < kTT; o += 256) {
      const int k = 2 * (o / (2 * kTB)) + (o & 1), l = (o % (2 * kTB)) / 2;
      double v = mode == 0 ? A[l][k] : A[k][l];
      if (slot == 0) v = (k == l ? 0.0 : v) * rds[l];
      dst[(size_t)slot * kTT + o] = v;
    }
  }
  if (mode == 0 && threadIdx.x < kTB) tiles[(size_t)2 * nbk * 3 * kTT + (size_t)i * kTB + threadIdx.x] = rds[threadIdx.x];
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

static size_t trsv_tiles_size(int64_t n) {
  const size_t nbk = (size_t)((n + kTB - 1) / kTB);
  return 2 * nbk * 3 * kTT + nbk * kTB;
}

void prepare_trsv(Problem& P) {
  const int nbk = (int)((P.n + kTB - 1) / kTB);
  P.d_trsv_tiles.resize(trsv_tiles_size(P.n));
  hipLaunchKernelGGL(k_trsv_tiles, dim3(nbk, 2), dim3(256), 0, P.stream, P.d_R.p, nbk, P.d_trsv_tiles.p);
  RFM_HIP(hipGetLastError());
}

// x = R^{-1} (y * yscale) or R^{-T} (y * yscale); with st != null the scale and the
// subtraction coefficient come from the LSQR state.  sub_vec may alias x.
void launch_trsv(Problem& P, const double* y, double* x, bool transpose, const double* sub_vec,
                 const LsqrState* st, int yscale_sel, int sub_sel, double* red_partials) {
  const int nbk = (int)((P.n + kTB - 1) / kTB);
  RFM_CHECK((int64_t)kTrsvErr < (int64_t)P.d_sync.n, RFM_EINVAL, "triangular solve: no sync words");
  RFM_CHECK(P.d_trsv_tiles.n >= trsv_tiles_size(P.n), RFM_EINVAL, "triangular solve: R has not been prepared");
  P.d_trsv.resize((size_t)2 * nbk * kTB);
  double* z = P.d_trsv.p;                     // published blocks of x, nbk * 64
  double* pz = P.d_trsv.p + (size_t)nbk * kTB;  // helper partials, nbk * 64
  const double nn = (double)P.n;
  const int64_t nz = 2 * (int64_t)nbk * kTB;  // z and pz are contiguous
  hipLaunchKernelGGL(k_trsv_clear, dim3((unsigned)((nz + 255) / 256)), dim3(256), 0, P.stream, z, nz);
  ProfScope ps(P.prof, P.stream, "trsv", nn * nn, 8.0 * (nn * (nn + 1) / 2 + 3 * nn));
  if (transpose)
    hipLaunchKernelGGL(k_trsv<1>, dim3(nbk + 1), dim3(512), 0, P.stream, P.d_R.p, P.d_trsv_tiles.p, (int)P.n, nbk, y, z, pz, x,
                       sub_vec, st, yscale_sel, sub_sel, red_partials, P.d_sync.p);
  else
    hipLaunchKernelGGL(k_trsv<0>, dim3(nbk + 1), dim3(512), 0, P.stream, P.d_R.p, P.d_trsv_tiles.p, (int)P.n, nbk, y, z, pz, x,
                       sub_vec, st, yscale_sel, sub_sel, red_partials, P.d_sync.p);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
