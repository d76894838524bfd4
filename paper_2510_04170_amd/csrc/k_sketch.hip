// Gaussian sketch B = S (D J) (the sketch of Sec. 4.1 taken Gaussian).
//
// S is never stored.  Entry S[i][r] is N(0,1)/sqrt(s) from Philox4x64-10
// (Salmon et al., SC'11) with counter (i/8, r, 0, 0) and key (seed, jac_index);
// each of the four 64-bit outputs is one Box-Muller pair (32-bit uniforms),
// giving the entries of rows 8q .. 8q+7.  Each Gaussian is drawn again for every
// 128-column tile of every column block its row touches (S is never stored).
// The logarithm and the cosine / sine of the pair are evaluated here from their
// series (atanh series of the mantissa, Taylor series after an exact quarter-turn
// reduction), to about 1 ulp, at half the instructions of the library calls.
//
// Work unit: one workgroup computes a 128 x 128 tile of B for one column block
// (box e, component c): sketch rows i0 .. i0+127 and block columns c0 .. c0+127.
// Its k loop runs over the block's list of Jacobian rows, 16 at a time (one
// ragged chunk per block, not one per tile): each of the 256 threads draws 8
// entries of the 128 x 16 slice of S with one Philox call and loads 8 entries
// of the 16 x 128 slice of D J, both into LDS, and four wavefronts (2 x 2)
// accumulate 64 x 64 blocks on v_mfma_f64_4x4x4_4b.  The next chunk's draws
// and loads are issued before the current chunk's MFMAs.  Workgroups are
// ordered so that each XCD runs the row tiles of one column tile together,
// and they read the same D J rows from its L2 at about the same time.
//
// Measured on gfx950, the draws' vector instructions and the MFMAs do not
// overlap: the kernel's time is the MFMA time plus the draw time (Philox's
// 64-bit multiplies are the larger part of the latter).
#include "mfma_f64.h"
#include "rfm_internal.h"

namespace rfm {

namespace {

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

// ln(h 2^-32) for an integer 1 <= h <= 2^32: h = m 2^e with m in [sqrt(1/2), sqrt(2)), so that
// ln = (e - 32) ln 2 + ln m and ln m = 2 atanh(t), t = (m - 1) / (m + 1), |t| <= 0.1716, summed as the
// odd series 2 (t + t^3/3 + ... + t^21/21) (the next term is below 1e-18 t).
__device__ __forceinline__ double bm_ln_fixed32(uint64_t h) {
  int e;
  double m = frexp((double)h, &e);  // h = m 2^e, m in [1/2, 1)
  if (m < 0.70710678118654752440) {
    m *= 2.0;
    e -= 1;
  }
  const double num = m - 1.0, den = m + 1.0;  // both exact: m has at most 32 significant bits
  double r = __builtin_amdgcn_rcp(den);
  r = fma(r, fma(-den, r, 1.0), r);
  r = fma(r, fma(-den, r, 1.0), r);
  double t = num * r;
  t = fma(r, fma(-den, t, num), t);
  const double t2 = t * t;
  double p = 1.0 / 21;
  p = fma(p, t2, 1.0 / 19);
  p = fma(p, t2, 1.0 / 17);
  p = fma(p, t2, 1.0 / 15);
  p = fma(p, t2, 1.0 / 13);
  p = fma(p, t2, 1.0 / 11);
  p = fma(p, t2, 1.0 / 9);
  p = fma(p, t2, 1.0 / 7);
  p = fma(p, t2, 1.0 / 5);
  p = fma(p, t2, 1.0 / 3);
  const double tt = 2.0 * t;
  const double lnm = fma(tt * t2, p, tt);
  return fma((double)(e - 32), 0.69314718055994530942, lnm);
}

// cos and sin of 2 pi lo 2^-32 for an integer 0 <= lo < 2^32: with q = nearest integer to lo 2^-30,
// the angle is (pi / 2) (q + r), r = lo 2^-30 - q in [-1/2, 1/2] exactly, theta = (pi / 2) r in
// [-pi/4, pi/4]; sin and cos of theta by their Taylor series to theta^17 and theta^18 (remainders
// below 1e-19), then rotated by q quarter turns.
__device__ __forceinline__ void bm_cossin_turn32(uint64_t lo, double* c, double* s) {
  const int64_t q = (int64_t)((lo + (1ull << 29)) >> 30);          // 0 .. 4
  const int64_t ri = (int64_t)lo - (q << 30);                        // -2^29 .. 2^29 - 1
  const double th = (double)ri * (3.14159265358979323846 / 2147483648.0);  // (pi / 2) ri 2^-30
  const double x2 = th * th;
  double ps = -1.0 / 355687428096000.0;          // -1/17!
  ps = fma(ps, x2, 1.0 / 1307674368000.0);       // 1/15!
  ps = fma(ps, x2, -1.0 / 6227020800.0);         // -1/13!
  ps = fma(ps, x2, 1.0 / 39916800.0);            // 1/11!
  ps = fma(ps, x2, -1.0 / 362880.0);             // -1/9!
  ps = fma(ps, x2, 1.0 / 5040.0);                // 1/7!
  ps = fma(ps, x2, -1.0 / 120.0);                // -1/5!
  ps = fma(ps, x2, 1.0 / 6.0);                   // 1/3! (sign folded below)
  const double sn = fma(-th * x2, ps, th);
  double pc = 1.0 / 6402373705728000.0;          // 1/18!
  pc = fma(pc, x2, -1.0 / 20922789888000.0);     // -1/16!
  pc = fma(pc, x2, 1.0 / 87178291200.0);         // 1/14!
  pc = fma(pc, x2, -1.0 / 479001600.0);          // -1/12!
  pc = fma(pc, x2, 1.0 / 3628800.0);             // 1/10!
  pc = fma(pc, x2, -1.0 / 40320.0);              // -1/8!
  pc = fma(pc, x2, 1.0 / 720.0);                 // 1/6!
  pc = fma(pc, x2, -1.0 / 24.0);                 // -1/4!
  pc = fma(pc, x2, 0.5);                         // 1/2! (sign folded below)
  const double cs = fma(-x2, pc, 1.0);
  const bool sw = q & 1;
  const double a = sw ? sn : cs, b = sw ? cs : sn;
  *c = ((q + 1) & 2) ? -a : a;
  *s = (q & 2) ? -b : b;
}

// Box-Muller on one 64-bit word: u1 = (hi + 1) 2^-32 in (0,1], u2 = lo 2^-32 in [0,1);
// z0, z1 = sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2)
__device__ __forceinline__ void box_muller(uint64_t x, double& z0, double& z1) {
  const double rad = sqrt(-2.0 * bm_ln_fixed32((x >> 32) + 1));
  double c, sn;
  bm_cossin_turn32(x & 0xFFFFFFFFull, &c, &sn);
  z0 = rad * c;
  z1 = rad * sn;
}

// Sketch rows r0 .. r0 + nr - 1 (r0 a multiple of 128) of B = S (D J) into out, sketch row r0 + i of
// column c at out[c ldo + i].  lb .. le: the block's rows in lrow / loff; nrt x nct tiles per block.
__global__ void __launch_bounds__(256, 2) k_sketch_f64(const int64_t* __restrict__ lptr,
                                                      const int32_t* __restrict__ lrow,
                                                      const int64_t* __restrict__ loff,
                                                      const double* __restrict__ Jv, int J, int64_t r0, int64_t nr,
                                                      int nrt, int nct, double inv_sqrt_s, uint64_t seed,
                                                      uint64_t jac, double* __restrict__ out, int64_t ldo) {
  __shared__ double Ss[2][kKC][kBig + 1];  // S tile [chunk row][sketch row]
  __shared__ double Ds[2][kKC][kBig + 1];  // D J tile [chunk row][column]
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int wr = wv / 2, wc = wv % 2;
  const int L = xcd_order(blockIdx.x, gridDim.x);
  const int rt = L % nrt, ct = (L / nrt) % nct, blk = L / nrt / nct;
  const int64_t i0 = r0 + (int64_t)rt * kBig, iend = r0 + nr;
  const int c0 = ct * kBig;
  const int64_t lb = lptr[blk], le = lptr[blk + 1];
  // wavefronts whose 64 x 64 block lies wholly past the last row or column skip the products
  const bool active = i0 + wr * 64 < iend && c0 + wc * 64 < J;
  // draw role: sketch rows 8 gq .. 8 gq + 7 of the tile at chunk row gk
  const int gq = tid % 16, gk = tid / 16;
  // load role: column lc at chunk rows lk + 2 t (lk is the same across a wavefront)
  const int lc = tid % kBig;
  const int lk = __builtin_amdgcn_readfirstlane(tid / kBig);
  const bool cin = c0 + lc < J;
  double z[8], dv[8];
  auto produce = [&](int64_t k0) {
    const int64_t e = k0 + gk;
    if (e < le) {
      uint64_t x0 = (uint64_t)(i0 / 8 + gq), x1 = (uint64_t)lrow[e], x2 = 0, x3 = 0;
      philox4x64_10(x0, x1, x2, x3, seed, jac);
      box_muller(x0, z[0], z[1]);
      box_muller(x1, z[2], z[3]);
      box_muller(x2, z[4], z[5]);
      box_muller(x3, z[6], z[7]);
#pragma unroll
      for (int t = 0; t < 8; ++t) z[t] *= inv_sqrt_s;
    } else {
#pragma unroll
      for (int t = 0; t < 8; ++t) z[t] = 0.0;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t e2 = k0 + lk + 2 * t;
      dv[t] = (e2 < le && cin) ? Jv[loff[e2] + c0 + lc] : 0.0;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int t = 0; t < 8; ++t) Ss[buf][gk][8 * gq + t] = z[t];
#pragma unroll
    for (int t = 0; t < 8; ++t) Ds[buf][lk + 2 * t][lc] = dv[t];
  };
  double acc[4][16];
#pragma unroll
  for (int rg = 0; rg < 4; ++rg)
#pragma unroll
    for (int cg = 0; cg < 16; ++cg) acc[rg][cg] = 0.0;
  if (lb < le) {
    produce(lb);
    stash(0);
  }
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = lb; k0 < le; k0 += kKC) {
    const bool more = k0 + kKC < le;
    if (more) produce(k0 + kKC);
    if (active) mfma4_chunk(Ss[buf], Ds[buf], lane, wr, wc, acc);
    if (more) stash(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  // acc[rg][cg] in lane l: tile row wr 64 + rg 16 + l % 16, tile column wc 64 + cg 4 + l / 16
#pragma unroll
  for (int cg = 0; cg < 16; ++cg) {
    const int col = c0 + wc * 64 + cg * 4 + lane / 16;
    if (col >= J) continue;
    double* bcol = out + ((int64_t)blk * J + col) * ldo - r0;
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) {
      const int64_t i = i0 + wr * 64 + rg * 16 + lane % 16;
      if (i < iend) bcol[i] = acc[rg][cg];
    }
  }
}

}  // namespace

void launch_sketch_rows(Problem& P, uint64_t seed, uint64_t jac_index, int64_t r0, int64_t nr, double* out,
                        int64_t ldo) {
  RFM_CHECK(r0 % kBig == 0 && nr >= 0 && r0 + nr <= P.s && ldo >= nr, RFM_EINVAL, "sketch: bad row range");
  if (nr == 0) return;
  const int nblk = P.geom.nbox * P.ncomp;
  const int nrt = (int)((nr + kBig - 1) / kBig), nct = (P.J + kBig - 1) / kBig;
  const int64_t nwg = (int64_t)nrt * nct * nblk;
  RFM_CHECK(nwg < (int64_t)INT32_MAX, RFM_EINVAL, "sketch: too many tiles");
  const double sq = 1.0 / sqrt((double)P.s);
  ProfScope ps(P.prof, P.stream, "sketch_f64", 2.0 * (double)nr * P.nvals, 8.0 * ((double)P.nvals + (double)nr * P.n));
  hipLaunchKernelGGL(k_sketch_f64, dim3((unsigned)nwg), dim3(256), 0, P.stream, P.d_sk_ptr.p, P.d_sk_row.p,
                     P.d_sk_off.p, P.d_J.p, P.J, r0, nr, nrt, nct, sq, seed, jac_index, out, ldo);
  RFM_HIP(hipGetLastError());
}

void launch_sketch(Problem& P, uint64_t seed, uint64_t jac_index, int prec) {
  (void)prec;  // the FP64 product; lower-precision products are selected in the solver
  P.d_B.resize((size_t)P.s * P.n);
  launch_sketch_rows(P, seed, jac_index, 0, P.s, P.d_B.p, P.s);
}

}  // namespace rfm
