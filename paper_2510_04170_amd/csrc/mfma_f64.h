// FP64 matrix-core building blocks shared by the QR trailing update and the
// Gaussian sketch: 128 x 128 output tiles, four wavefronts in a 2 x 2
// arrangement each owning 64 x 64 outputs (64 accumulators per lane) on
// v_mfma_f64_4x4x4_4b_f64, operands staged through LDS 16 values of k at a time.
#pragma once

#include <hip/hip_runtime.h>

namespace rfm {

constexpr int kBig = 128;
constexpr int kKC = 16;

typedef double v2d __attribute__((ext_vector_type(2)));

// Workgroups are dealt to the 8 XCDs round robin (workgroup id mod 8), and each XCD has its own L2.
// The position of workgroup `id` in a sequence where every XCD takes a contiguous range, so that
// workgroups that share operands can be placed on one XCD and run there close in time.
__device__ __forceinline__ int xcd_order(int id, int total) {
  const int per = total / 8, x = id % 8, q = id / 8;
  return q < per ? x * per + q : 8 * per + x;
}

// One 16-deep k-chunk on LDS tiles Xs[k][row], Ys[k][col] (row and column of the output; LDX and LDY
// are the padded widths of the two tiles).
// v_mfma_f64_4x4x4_4b_f64 holds, for block b, A(i,k) in lane 16k+4b+i, B(k,j) in lane 16k+4b+j
// and D(i,j) in lane 16i+4b+j.  With the A operand carrying 4 output columns (the same in every
// block) and the B operand 16 output rows, acc[rg][cg] in lane l is output row rg*16 + l%16 and
// column cg*4 + l/16 of the wavefront's 64 x 64 block: 16 consecutive rows of one column per
// 16 lanes, which suits column-major stores.
template <int LDX, int LDY>
__device__ __forceinline__ void mfma4_chunk(const double (*Xs)[LDX], const double (*Ys)[LDY], int lane, int wr,
                                            int wc, double (&acc)[4][16]) {
#pragma unroll
  for (int ks = 0; ks < kKC / 4; ++ks) {
    const int kr = ks * 4 + lane / 16;
    double x[4];
#pragma unroll
    for (int rg = 0; rg < 4; ++rg) x[rg] = Xs[kr][wr * 64 + rg * 16 + lane % 16];
    // the column operands in two halves keep the kernel within 256 VGPRs
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double y[8];
#pragma unroll
      for (int cg = 0; cg < 8; ++cg) y[cg] = Ys[kr][wc * 64 + (h * 8 + cg) * 4 + lane % 4];
#pragma unroll
      for (int rg = 0; rg < 4; ++rg)
#pragma unroll
        for (int cg = 0; cg < 8; ++cg)
          acc[rg][h * 8 + cg] = __builtin_amdgcn_mfma_f64_4x4x4f64(y[cg], x[rg], acc[rg][h * 8 + cg], 0, 0, 0);
    }
  }
}

}  // namespace rfm
