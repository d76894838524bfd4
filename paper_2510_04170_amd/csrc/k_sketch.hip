// Gaussian sketch B = S (D J) (the sketch of Sec. 4.1 taken Gaussian).
//
// S is never stored.  Entry S[i][r] is N(0,1)/sqrt(s) from Philox4x64-10
// (Salmon et al., SC'11) with counter (i/8, r, 0, 0) and key (seed, jac_index);
// each of the four 64-bit outputs is one Box-Muller pair (32-bit uniforms),
// giving the entries of rows 8q .. 8q+7.  Because every Jacobian row touches at
// most two column blocks, each Gaussian is generated once per column block it
// meets.
//
// Work unit: one workgroup computes a 64-row x J-column slab of B for one
// column block (box e, component c) and runs over every stored Jacobian tile
// that touches the block.  Per 32-row chunk of those tiles, the 256 threads
// generate the 64 x 32 slice of S into LDS (one Philox call each), and each
// wavefront accumulates its column tiles with v_mfma_f64_16x16x4 from the
// Jacobian rows read straight from HBM.
#include "rfm_internal.h"

namespace rfm {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr uint64_t kM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kM1 = 0xCA5A826395121157ull;
constexpr uint64_t kW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox4x64_10(uint64_t& c0, uint64_t& c1, uint64_t& c2, uint64_t& c3, uint64_t k0,
                                              uint64_t k1) {
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint64_t hi0 = __umul64hi(kM0, c0), lo0 = kM0 * c0;
    const uint64_t hi1 = __umul64hi(kM1, c2), lo1 = kM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0;
    const uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
}

// Box-Muller on one 64-bit word: u1 = (hi + 1) 2^-32 in (0,1], u2 = lo 2^-32 in [0,1);
// cos/sin(2 pi u2) as cospi/sinpi(2 u2), whose argument needs no range reduction
__device__ __forceinline__ void box_muller(uint64_t x, double& z0, double& z1) {
  const double u1 = ((double)(x >> 32) + 1.0) * 0x1.0p-32;
  const double u2 = (double)(x & 0xFFFFFFFFull) * 0x1.0p-32;
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  z0 = rad * cs;
  z1 = rad * sn;
}

constexpr int kSRows = 64;   // sketch rows per workgroup
constexpr int kChunk = 32;   // Jacobian rows per LDS stage

// NCTW: 16-column MFMA tiles per wavefront (wavefront w owns tiles w, w+4, ...)
template <int NCTW>
__global__ void __launch_bounds__(256) k_sketch_f64(const TileDesc* __restrict__ tiles,
                                                    const int32_t* __restrict__ cb_ptr,
                                                    const int32_t* __restrict__ cb_tile,
                                                    const int32_t* __restrict__ cb_off,
                                                    const double* __restrict__ Jv, int J, int64_t s,
                                                    double inv_sqrt_s, uint64_t seed, uint64_t jac,
                                                    double* __restrict__ B) {
  __shared__ double sS[kChunk][kSRows + 1];
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int64_t i0 = (int64_t)blockIdx.x * kSRows;
  const int blk = blockIdx.y;
  const int ntc = (J + 15) / 16;

  v4d acc[4][NCTW];
#pragma unroll
  for (int rt = 0; rt < 4; ++rt)
#pragma unroll
    for (int k = 0; k < NCTW; ++k) acc[rt][k] = v4d{0, 0, 0, 0};

  // generation role of this thread: sketch rows 8*qi .. 8*qi+7 of the slab, Jacobian row rr of the chunk
  const int qi = tid % 8, rr = tid / 8;

  for (int kk = cb_ptr[blk]; kk < cb_ptr[blk + 1]; ++kk) {
    const TileDesc td = tiles[cb_tile[kk]];
    const int off = cb_off[kk];
    const int w = td.wA + td.wB;
    for (int base = 0; base < td.nrows; base += kChunk) {
      // S[i0 .. i0+63][row0+base .. +31] into LDS
      {
        const int rloc = base + rr;
        double z[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (rloc < td.nrows) {
          uint64_t c0 = (uint64_t)(i0 / 8 + qi), c1 = (uint64_t)(td.row0 + rloc), c2 = 0, c3 = 0;
          philox4x64_10(c0, c1, c2, c3, seed, jac);
          box_muller(c0, z[0], z[1]);
          box_muller(c1, z[2], z[3]);
          box_muller(c2, z[4], z[5]);
          box_muller(c3, z[6], z[7]);
#pragma unroll
          for (int t = 0; t < 8; ++t) z[t] *= inv_sqrt_s;
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) sS[rr][8 * qi + t] = z[t];
      }
      __syncthreads();
#pragma unroll
      for (int ks = 0; ks < kChunk / 4; ++ks) {
        const int kr = ks * 4 + lane / 16;  // chunk row of this lane's operands
        const bool rvalid = base + kr < td.nrows;
        double a[4];
#pragma unroll
        for (int rt = 0; rt < 4; ++rt) a[rt] = sS[kr][rt * 16 + lane % 16];
        const double* jrow = Jv + td.val_off + (int64_t)(base + kr) * w + off;
#pragma unroll
        for (int k = 0; k < NCTW; ++k) {
          const int ct = wv + 4 * k;
          const int col = ct * 16 + lane % 16;
          double bv = 0.0;
          if (ct < ntc && col < J && rvalid) bv = jrow[col];
#pragma unroll
          for (int rt = 0; rt < 4; ++rt) acc[rt][k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rt], bv, acc[rt][k], 0, 0, 0);
        }
      }
      __syncthreads();
    }
  }
  // store: v_mfma_f64_16x16x4 leaves row (l/16) + 4t, column l%16 of the tile in lane l, element t
#pragma unroll
  for (int k = 0; k < NCTW; ++k) {
    const int ct = wv + 4 * k;
    const int col = ct * 16 + lane % 16;
    if (ct >= ntc || col >= J) continue;
    double* bcol = B + ((int64_t)blk * J + col) * s;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t i = i0 + rt * 16 + (lane / 16) + 4 * t;
        if (i < s) bcol[i] = acc[rt][k][t];
      }
  }
}

}  // namespace

void launch_sketch(Problem& P, uint64_t seed, uint64_t jac_index, int prec) {
  (void)prec;  // the FP64 product; lower-precision products are selected in the solver
  const size_t need = (size_t)P.s * P.n;
  P.d_B.resize(need);
  const int nblk = P.geom.nbox * P.ncomp;
  dim3 grid((unsigned)((P.s + kSRows - 1) / kSRows), (unsigned)nblk);
  const int ntc = (P.J + 15) / 16;
  const int nctw = (ntc + 3) / 4;
  const double sq = 1.0 / sqrt((double)P.s);
  ProfScope ps(P.prof, P.stream, "sketch_f64", 2.0 * (double)P.s * P.nvals, 8.0 * ((double)P.nvals + (double)P.s * P.n));
  switch (nctw) {
#define RFM_CASE(N)                                                                                          \
  case N:                                                                                                    \
    hipLaunchKernelGGL(k_sketch_f64<N>, grid, dim3(256), 0, P.stream, P.d_tiles.p, P.d_cb_ptr.p, P.d_cb_tile.p, \
                       P.d_cb_off.p, P.d_J.p, P.J, P.s, sq, seed, jac_index, P.d_B.p);                        \
    break;
    RFM_CASE(1) RFM_CASE(2) RFM_CASE(3) RFM_CASE(4) RFM_CASE(5) RFM_CASE(6) RFM_CASE(7) RFM_CASE(8)
#undef RFM_CASE
    default:
      throw Error(RFM_EINVAL, "sketch: J above 512");
  }
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
