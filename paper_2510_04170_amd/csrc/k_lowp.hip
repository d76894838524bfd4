// Low-precision forms of the sketch (Sec. 4.1) and of the LSQR operator.
//
// The preconditioner only has to embed the column space of D J, but a
// perturbation E of D J lifts the small singular values of the sketch to about
// ||E||, and D J R^-1 then has singular values down to sigma_min(D J) / ||E||.
// With kappa(D J) up to ~1e13 the operand must keep ~40 bits and the sums must
// not round.  So D J is cut into integer pieces on a fixed-point grid per
// (column, chunk of at most 128 rows): E = floor(log2 max|D J|) + 1 over the
// chunk, q_p = nearest integer to X_p / 2^(E - b(p+1)) with b = 8 (BF16) or 4
// (FP8), X_{p+1} = X_p - q_p 2^(E - b(p+1)).  S is an integer code K[b] / k_s
// (k_s = 32 for BF16, 4 for FP8).  Every matrix-core sum over a chunk is then
// an integer (BF16: |sum| <= 128 * 92 * 256 < 2^24) or a multiple of 2^-8 below
// 2^15 (FP8, three pieces at once through the E8M0 operand scales 2^0, 2^-4,
// 2^-8), so the FP32 accumulator never rounds; the chunk results are scaled by
// powers of two and summed in FP64.  Six BF16 or twelve FP8 pieces keep 48
// bits of each chunk's largest entry.
//
// S codes: entry S[i][r] uses byte (i mod 32) of the Philox4x64-10 block for
// counter (i / 32, r, 1, 0) and key (seed, jac_index); K[b] is the integer
// nearest to k_s Phi^-1((b + 1/2) / 256).  One generator call yields 32 codes.
//
// Operand layout ("panels"): for each column block (box e, component c), the
// 32-row groups of global rows that touch it, ascending, padded with empty
// groups to a multiple of four; chunk h is slots 4h .. 4h+3.  Slot k of a
// group holds row 32 g + k.  A piece is stored [slot][column][32 rows]: for
// v_mfma_f32_16x16x32_bf16 lane (q, c) reads rows 8q .. 8q+7 of one slot; for
// v_mfma_scale_f32_16x16x128_f8f6f4 (one chunk per instruction) lane (q, c)
// reads rows 16(q%2) .. +15 of slots q/2 and 2 + q/2.
#include "rfm_internal.h"

#include <cmath>
#include <type_traits>

namespace rfm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef int v8i __attribute__((ext_vector_type(8)));

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

// ---------------------------------------------------------------------------
// encodings of small integers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint16_t bf16_bits_int(double q) {  // |q| <= 256, an integer
  return (uint16_t)(__float_as_uint((float)q) >> 16);
}

// OCP E4M3 code of an integer |q| <= 16 (4 significant bits, bias 7)
__device__ __forceinline__ uint8_t e4m3_bits_int(double q) {
  if (q == 0.0) return 0;
  const uint8_t sgn = q < 0 ? 0x80 : 0;
  int e;
  const double f = frexp(fabs(q), &e);  // |q| = f 2^e, f in [0.5, 1)
  return sgn | (uint8_t)((e - 1 + 7) << 3) | (uint8_t)((int)(f * 16.0) - 8);
}

// ---------------------------------------------------------------------------
// casts
// ---------------------------------------------------------------------------

// one thread per (chunk, column): E from the chunk's largest entry, then the
// pieces of each slot's 32 rows.  BITS = 8 (BF16 codes) or 4 (E4M3 codes).
template <int BITS, typename TC>
__global__ void __launch_bounds__(256) k_cast_fixed(const int64_t* __restrict__ slot_rowoff, int64_t nchunks, int J,
                                                    const double* __restrict__ Jv, int npc, int64_t piece_stride,
                                                    TC* __restrict__ out, int32_t* __restrict__ pexp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nchunks * J) return;
  const int64_t ch = t / J;
  const int col = (int)(t - ch * J);
  const int64_t* ro = slot_rowoff + ch * 128;
  double mx = 0.0;
  for (int k = 0; k < 128; ++k) {
    const int64_t off = ro[k];
    if (off >= 0) mx = fmax(mx, fabs(Jv[off + col]));
  }
  int E = 0;
  if (mx > 0.0) (void)frexp(mx, &E);  // mx = f 2^E, f in [0.5, 1)
  pexp[t] = E;
  constexpr int PER_WORD = 4 / sizeof(TC);  // codes per 32-bit word
  constexpr int WORDS = 32 / PER_WORD;      // words per slot and piece
  for (int sl = 0; sl < 4; ++sl) {
    double x[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const int64_t off = ro[32 * sl + k];
      x[k] = off >= 0 ? Jv[off + col] : 0.0;
    }
    const int64_t slot = ch * 4 + sl;
    for (int p = 0; p < npc; ++p) {
      const int sh = E - BITS * (p + 1);
      uint32_t w[WORDS];
#pragma unroll
      for (int v = 0; v < WORDS; ++v) w[v] = 0;
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const double q = rint(ldexp(x[k], -sh));
        x[k] -= ldexp(q, sh);
        const uint32_t code = sizeof(TC) == 2 ? (uint32_t)bf16_bits_int(q) : (uint32_t)e4m3_bits_int(q);
        w[k / PER_WORD] |= code << (8 * sizeof(TC) * (k % PER_WORD));
      }
      uint4* d4 = reinterpret_cast<uint4*>(out + p * piece_stride + (slot * J + col) * 32);
#pragma unroll
      for (int v = 0; v < WORDS / 4; ++v) d4[v] = make_uint4(w[4 * v], w[4 * v + 1], w[4 * v + 2], w[4 * v + 3]);
    }
  }
}

__global__ void k_cast_f32(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (float)x[i];
}

// ---------------------------------------------------------------------------
// the sketch products
// ---------------------------------------------------------------------------

constexpr int kRowsWG = 128;  // sketch rows per workgroup: two wavefront rows of 64
constexpr int kColsWG = 160;  // columns per workgroup: two wavefront columns of 80
constexpr int kCT = 5;        // 16-column tiles per wavefront
constexpr int kRT = 4;        // 16-row tiles per wavefront

// codes S[i0 + 32 q + t][chunk row k] into LDS: thread (q = wavefront, k = lane + 64 j) makes one
// generator call per chunk row it owns and looks its 32 bytes up in the code table
template <typename TS, int LDW>
__device__ __forceinline__ void gen_chunk(TS (*sS)[LDW], const TS* __restrict__ tab, const int32_t* __restrict__ sgrp,
                                          int64_t slot0, int64_t i0, uint64_t seed, uint64_t jac) {
  const int q = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int k = lane + 64 * j;
    const int g = sgrp[slot0 + k / 32];
    TS z[32];
    if (g >= 0) {
      uint64_t c0 = (uint64_t)(i0 / 32 + q), c1 = (uint64_t)g * 32 + (k % 32), c2 = 1, c3 = 0;
      philox4x64_10(c0, c1, c2, c3, seed, jac);
      const uint64_t wd[4] = {c0, c1, c2, c3};
#pragma unroll
      for (int t = 0; t < 32; ++t) z[t] = tab[(wd[t / 8] >> (8 * (t % 8))) & 0xFF];
    } else {
#pragma unroll
      for (int t = 0; t < 32; ++t) z[t] = 0;
    }
#pragma unroll
    for (int t = 0; t < 32; ++t) sS[32 * q + t][k] = z[t];
  }
}

// B[:, block columns] for one 128-row slab and up to 160 columns of one column block
template <bool FP8>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) k_sketch_fixed(const int32_t* __restrict__ cbs_ptr,
                                                      const int32_t* __restrict__ slot_group,
                                                      const void* __restrict__ pan_, const int32_t* __restrict__ pexp,
                                                      int64_t piece_stride, int npc, int J, int64_t r0,
                                                      int64_t nr, double inv_scale, uint64_t seed, uint64_t jac,
                                                      const void* __restrict__ table_, double* __restrict__ out,
                                                      int64_t ldo) {
  typedef typename std::conditional<FP8, uint8_t, uint16_t>::type TC;
  constexpr int LDW = FP8 ? 128 + 16 : 128 + 8;
  constexpr int BITS = FP8 ? 4 : 8;
  __shared__ __attribute__((aligned(16))) TC sS[kRowsWG][LDW];
  __shared__ __attribute__((aligned(16))) TC tab[256];
  const TC* pan = reinterpret_cast<const TC*>(pan_);
  const int tid = threadIdx.x, lane = tid % 64, wv = tid / 64;
  const int wr = wv / 2, wc = wv % 2;
  const int q = lane / 16, c16 = lane % 16;
  const int64_t i0 = r0 + (int64_t)blockIdx.x * kRowsWG, iend = r0 + nr;
  const int blk = blockIdx.y;
  const int colw = blockIdx.z * kColsWG + wc * 80;
  tab[tid] = reinterpret_cast<const TC*>(table_)[tid];
  const int64_t sbeg = cbs_ptr[blk];
  const int nch = (cbs_ptr[blk + 1] - cbs_ptr[blk]) / 4;

  double acc[kRT][kCT][4];
#pragma unroll
  for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
    for (int tc = 0; tc < kCT; ++tc)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[rt][tc][t] = 0.0;

  for (int ch = 0; ch < nch; ++ch) {
    const int64_t slot0 = sbeg + 4 * ch;
    __syncthreads();  // previous chunk's reads of sS are done (and tab is in place)
    gen_chunk<TC, LDW>(sS, tab, slot_group, slot0, i0, seed, jac);
    __syncthreads();
    int ex[kCT], colc[kCT];
#pragma unroll
    for (int tc = 0; tc < kCT; ++tc) {
      const int col = colw + 16 * tc + c16;
      colc[tc] = col < J ? col : J - 1;
      ex[tc] = pexp[(slot0 / 4) * J + colc[tc]];
    }
    if constexpr (!FP8) {
      for (int p = 0; p < npc; ++p) {
        v4f a32[kRT][kCT];
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc) a32[rt][tc] = v4f{0, 0, 0, 0};
        // B fragments one k-step ahead of the products that use them (five loads in flight while
        // twenty products run); a column past J reads column J - 1 instead, which only feeds output
        // columns that are never stored
        const TC* pb = pan + p * piece_stride + 8 * q;
        // re-read the A fragments from LDS in every piece (keeps 64 registers free for loads in flight
        // instead of holding the piece-invariant fragments across the loop)
        int aoff = (wr * 64 + c16) * LDW + 8 * q;
        asm volatile("" : "+v"(aoff));
        uint4 bn[kCT];
#pragma unroll
        for (int tc = 0; tc < kCT; ++tc) bn[tc] = *reinterpret_cast<const uint4*>(pb + (slot0 * J + colc[tc]) * 32);
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
          uint4 bc[kCT];
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc) bc[tc] = bn[tc];
          if (ks < 3) {
#pragma unroll
            for (int tc = 0; tc < kCT; ++tc)
              bn[tc] = *reinterpret_cast<const uint4*>(pb + ((slot0 + ks + 1) * J + colc[tc]) * 32);
          }
          __builtin_amdgcn_sched_barrier(0);  // keep the next k-step's loads ahead of these products
          v8bf a[kRT];
#pragma unroll
          for (int rt = 0; rt < kRT; ++rt)
            a[rt] = __builtin_bit_cast(v8bf, *reinterpret_cast<const uint4*>(&sS[0][0] + aoff + rt * 16 * LDW + 32 * ks));
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc) {
            const v8bf b = __builtin_bit_cast(v8bf, bc[tc]);
#pragma unroll
            for (int rt = 0; rt < kRT; ++rt)
              a32[rt][tc] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[rt], b, a32[rt][tc], 0, 0, 0);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int tc = 0; tc < kCT; ++tc) {
          const double sc = ldexp(inv_scale, ex[tc] - BITS * (p + 1));
#pragma unroll
          for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[rt][tc][t] += (double)a32[rt][tc][t] * sc;
        }
      }
    } else {
      v8i a[kRT];
#pragma unroll
      for (int rt = 0; rt < kRT; ++rt) {
        const TC* row = &sS[wr * 64 + rt * 16 + c16][0];
        const uint4 lo = *reinterpret_cast<const uint4*>(row + 16 * q);
        const uint4 hi = *reinterpret_cast<const uint4*>(row + 64 + 16 * q);
        a[rt] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
      for (int p0 = 0; p0 < npc; p0 += 3) {
        v4f a32[kRT][kCT];
#pragma unroll
        for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc) a32[rt][tc] = v4f{0, 0, 0, 0};
        const int pend = p0 + 3 < npc ? p0 + 3 : npc;
        for (int p = p0; p < pend; ++p) {
          const int scb = 127 - BITS * (p - p0);  // E8M0 2^(-4 (p - p0))
          v8i b[kCT];
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc) {
            const TC* base = pan + p * piece_stride;
            const uint4 lo = *reinterpret_cast<const uint4*>(base + ((slot0 + q / 2) * J + colc[tc]) * 32 + 16 * (q % 2));
            const uint4 hi =
                *reinterpret_cast<const uint4*>(base + ((slot0 + 2 + q / 2) * J + colc[tc]) * 32 + 16 * (q % 2));
            b[tc] = v8i{(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w, (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
          }
          __builtin_amdgcn_sched_barrier(0);  // all ten loads of this piece in flight before its products
#pragma unroll
          for (int tc = 0; tc < kCT; ++tc)
#pragma unroll
            for (int rt = 0; rt < kRT; ++rt)
              a32[rt][tc] =
                  __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a[rt], b[tc], a32[rt][tc], 0, 0, 0, 127, 0, scb);
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int tc = 0; tc < kCT; ++tc) {
          const double sc = ldexp(inv_scale, ex[tc] - BITS * (p0 + 1));
#pragma unroll
          for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
            for (int t = 0; t < 4; ++t) acc[rt][tc][t] += (double)a32[rt][tc][t] * sc;
        }
      }
    }
  }
  // lane (q, c) holds rows 4q + t of each 16 x 16 tile, column c
#pragma unroll
  for (int tc = 0; tc < kCT; ++tc) {
    const int col = colw + 16 * tc + c16;
    if (col >= J) continue;
    double* bcol = out + ((int64_t)blk * J + col) * ldo - r0;
#pragma unroll
    for (int rt = 0; rt < kRT; ++rt)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int64_t i = i0 + wr * 64 + rt * 16 + 4 * q + t;
        if (i < iend) bcol[i] = acc[rt][tc][t];
      }
  }
}

int default_pieces(int prec) { return prec == RFM_PREC_BF16 ? 6 : 12; }

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

// standard normal quantile by bisection on Phi(x) = erfc(-x / sqrt 2) / 2
static double normal_quantile(double p) {
  double lo = -40.0, hi = 40.0;
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid == lo || mid == hi) break;
    if (0.5 * std::erfc(-mid / std::sqrt(2.0)) < p)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

static uint8_t host_e4m3_int(double q) {  // E4M3 code of an integer |q| <= 16
  if (q == 0.0) return 0;
  const uint8_t sgn = q < 0 ? 0x80 : 0;
  int e;
  const double f = std::frexp(std::fabs(q), &e);
  return sgn | (uint8_t)((e - 1 + 7) << 3) | (uint8_t)((int)(f * 16.0) - 8);
}

// K[b] = nearest integer (ties to even) to k_s Phi^-1((b + 1/2) / 256)
void sketch_table(int prec, double* out) {
  const double ks = prec == RFM_PREC_BF16 ? 32.0 : 4.0;
  for (int b = 0; b < 256; ++b) out[b] = std::nearbyint(ks * normal_quantile((b + 0.5) / 256.0));
}

static void upload_tables(Problem& P) {
  if (P.have_tables) return;
  double t[256];
  std::vector<uint16_t> tb(256);
  sketch_table(RFM_PREC_BF16, t);
  for (int b = 0; b < 256; ++b) {
    const float f = (float)t[b];
    uint32_t u;
    std::memcpy(&u, &f, 4);
    tb[b] = (uint16_t)(u >> 16);
  }
  std::vector<uint8_t> t8(256);
  sketch_table(RFM_PREC_FP8, t);
  for (int b = 0; b < 256; ++b) t8[b] = host_e4m3_int(t[b]);
  P.d_tab16.resize(256);
  P.d_tab8.resize(256);
  RFM_HIP(hipMemcpy(P.d_tab16.p, tb.data(), 512, hipMemcpyHostToDevice));
  RFM_HIP(hipMemcpy(P.d_tab8.p, t8.data(), 256, hipMemcpyHostToDevice));
  P.have_tables = true;
}

void launch_cast_panels(Problem& P, int prec, int pieces) {
  upload_tables(P);
  const int npc = pieces > 0 ? pieces : default_pieces(prec);
  RFM_CHECK(npc >= 1 && npc <= kMaxPieces, RFM_EINVAL, "sketch pieces must be 1..16");
  const int64_t nchunks = P.nslots / 4;
  const int64_t per_piece = P.nslots * (int64_t)P.J * 32;  // codes of one piece
  const int64_t nthr = nchunks * (int64_t)P.J;
  const unsigned grid = (unsigned)((nthr + 255) / 256);
  P.d_pexp.resize((size_t)std::max<int64_t>(1, nthr));
  if (prec == RFM_PREC_BF16) {
    P.d_pan16.resize((size_t)npc * per_piece);
    ProfScope ps(P.prof, P.stream, "cast_bf16", 0.0, 16.0 * (double)P.nvals + 2.0 * npc * (double)per_piece);
    hipLaunchKernelGGL((k_cast_fixed<8, uint16_t>), dim3(grid), dim3(256), 0, P.stream, P.d_slot_rowoff.p, nchunks,
                       P.J, P.d_J.p, npc, per_piece, P.d_pan16.p, P.d_pexp.p);
  } else {
    P.d_pan8.resize((size_t)npc * per_piece);
    ProfScope ps(P.prof, P.stream, "cast_fp8", 0.0, 16.0 * (double)P.nvals + (double)npc * per_piece);
    hipLaunchKernelGGL((k_cast_fixed<4, uint8_t>), dim3(grid), dim3(256), 0, P.stream, P.d_slot_rowoff.p, nchunks,
                       P.J, P.d_J.p, npc, per_piece, P.d_pan8.p, P.d_pexp.p);
  }
  RFM_HIP(hipGetLastError());
  P.pan_prec = prec;
  P.pan_pieces = npc;
}

void launch_cast_f32(Problem& P) {
  P.d_J32.resize(P.nvals);
  ProfScope ps(P.prof, P.stream, "cast_f32", 0.0, 12.0 * (double)P.nvals);
  hipLaunchKernelGGL(k_cast_f32, dim3((unsigned)((P.nvals + 255) / 256)), dim3(256), 0, P.stream, P.d_J.p, P.nvals,
                     P.d_J32.p);
  RFM_HIP(hipGetLastError());
  P.have_J32 = true;
}

void launch_sketch_lowp_rows(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int64_t r0, int64_t nr,
                             double* out, int64_t ldo) {
  RFM_CHECK(prec == RFM_PREC_BF16 || prec == RFM_PREC_FP8, RFM_EINVAL, "sketch precision must be BF16 or FP8");
  RFM_CHECK(P.pan_prec == prec, RFM_EINVAL, "sketch: the operand pieces are not formed");
  RFM_CHECK(r0 % kRowsWG == 0 && nr >= 0 && r0 + nr <= P.s && ldo >= nr, RFM_EINVAL, "sketch: bad row range");
  if (nr == 0) return;
  const int npc = P.pan_pieces;
  const int nblk = P.geom.nbox * P.ncomp;
  dim3 grid((unsigned)((nr + kRowsWG - 1) / kRowsWG), (unsigned)nblk, (unsigned)((P.J + kColsWG - 1) / kColsWG));
  const double ks = prec == RFM_PREC_BF16 ? 32.0 : 4.0;
  const double inv_scale = 1.0 / (ks * std::sqrt((double)P.s));
  const int64_t per_piece = P.nslots * (int64_t)P.J * 32;
  // algorithmic work 2 s nnz(J) (the matrix cores issue every piece on the padded row chunks on top of it);
  // bytes: pieces once, B once
  const double flops = 2.0 * (double)nr * (double)P.nvals;
  const double bytes = (prec == RFM_PREC_BF16 ? 2.0 : 1.0) * npc * (double)per_piece + 8.0 * (double)nr * P.n;
  if (prec == RFM_PREC_BF16) {
    ProfScope ps(P.prof, P.stream, "sketch_bf16", flops, bytes);
    hipLaunchKernelGGL(k_sketch_fixed<false>, grid, dim3(256), 0, P.stream, P.d_cbs_ptr.p, P.d_slot_group.p,
                       (const void*)P.d_pan16.p, P.d_pexp.p, per_piece, npc, P.J, r0, nr, inv_scale, seed, jac_index,
                       (const void*)P.d_tab16.p, out, ldo);
  } else {
    ProfScope ps(P.prof, P.stream, "sketch_fp8", flops, bytes);
    hipLaunchKernelGGL(k_sketch_fixed<true>, grid, dim3(256), 0, P.stream, P.d_cbs_ptr.p, P.d_slot_group.p,
                       (const void*)P.d_pan8.p, P.d_pexp.p, per_piece, npc, P.J, r0, nr, inv_scale, seed, jac_index,
                       (const void*)P.d_tab8.p, out, ldo);
  }
  RFM_HIP(hipGetLastError());
}

void launch_sketch_lowp(Problem& P, uint64_t seed, uint64_t jac_index, int prec, int pieces) {
  RFM_CHECK(prec == RFM_PREC_BF16 || prec == RFM_PREC_FP8, RFM_EINVAL, "sketch precision must be BF16 or FP8");
  launch_cast_panels(P, prec, pieces);
  P.d_B.resize((size_t)P.s * P.n);
  launch_sketch_lowp_rows(P, seed, jac_index, prec, 0, P.s, P.d_B.p, P.s);
}

void get_sketch_operand(Problem& P, int piece, int blk, int64_t slot0, int64_t nslots, double* out, int32_t* groups,
                        int32_t* scale_exp) {
  RFM_CHECK(P.pan_prec == RFM_PREC_BF16 || P.pan_prec == RFM_PREC_FP8, RFM_EINVAL,
            "no low-precision sketch operand has been formed");
  RFM_CHECK(piece >= 0 && piece < P.pan_pieces, RFM_EINVAL, "piece index out of range");
  const int nblk = P.geom.nbox * P.ncomp;
  RFM_CHECK(blk >= 0 && blk < nblk, RFM_EINVAL, "column block out of range");
  const int64_t b0 = P.cbs_ptr_h[blk], nb = P.cbs_ptr_h[blk + 1] - b0;
  RFM_CHECK(slot0 >= 0 && nslots >= 0 && slot0 + nslots <= nb, RFM_EINVAL, "slot range out of range");
  const int J = P.J;
  const int bits = P.pan_prec == RFM_PREC_BF16 ? 8 : 4;
  const int64_t per_piece = P.nslots * (int64_t)J * 32;
  const int64_t cnt = nslots * J * 32;
  RFM_HIP(hipStreamSynchronize(P.stream));
  const int64_t nthr = (P.nslots / 4) * (int64_t)J;
  std::vector<int32_t> ex(nthr);
  RFM_HIP(hipMemcpy(ex.data(), P.d_pexp.p, nthr * 4, hipMemcpyDeviceToHost));
  std::vector<double> code(cnt);
  if (P.pan_prec == RFM_PREC_BF16) {
    std::vector<uint16_t> h(cnt);
    RFM_HIP(hipMemcpy(h.data(), P.d_pan16.p + piece * per_piece + (b0 + slot0) * J * 32, cnt * 2,
                      hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < cnt; ++i) {
      const uint32_t u = (uint32_t)h[i] << 16;
      float f;
      std::memcpy(&f, &u, 4);
      code[i] = f;
    }
  } else {
    std::vector<uint8_t> h(cnt);
    RFM_HIP(hipMemcpy(h.data(), P.d_pan8.p + piece * per_piece + (b0 + slot0) * J * 32, cnt, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < cnt; ++i) {
      const uint8_t c = h[i];
      const int e = (c >> 3) & 0xF, mt = c & 7;
      double v = e == 0 ? mt * 0x1p-9 : std::ldexp(1.0 + mt / 8.0, e - 7);
      code[i] = (c & 0x80) ? -v : v;
    }
  }
  for (int64_t k = 0; k < nslots; ++k) {
    const int64_t slot = b0 + slot0 + k;
    if (groups) groups[k] = P.slot_group_h[slot];
    for (int j = 0; j < J; ++j) {
      const int E = ex[(slot / 4) * J + j];
      if (scale_exp) scale_exp[k * J + j] = E;
      for (int r = 0; r < 32; ++r) {
        const int64_t i = (k * J + j) * 32 + r;
        out[i] = std::ldexp(code[i], E - bits * (piece + 1));
      }
    }
  }
}

}  // namespace rfm
