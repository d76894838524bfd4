// Coordinate network for the learned initial guess: a tanh multilayer
// perceptron  in -> width (tanh) -> ... -> width (tanh) -> out  (linear last
// layer), trained by mean-squared error with Adam (Kingma & Ba, ICLR 2015,
// Algorithm 1) on fields produced by the solver itself.
//
// Storage: FP32 master parameters (layer l: W_l [dout][din] row-major, then
// b_l [dout]) and Adam moments; for the matrix cores, BF16 copies of every
// W_l padded to K = 32 multiples, W_l [dout][Kp] and its transpose
// Wt_l [din][Np].  Precision modes:
//   RFM_PREC_BF16: the products h W^T and delta W run on
//     v_mfma_f32_16x16x32_bf16 (operands rounded to BF16, FP32 accumulation);
//   RFM_PREC_F32: the same products in FP32 on the vector units (a checking
//     mode).
// Weight gradients (sums over the batch) and everything elementwise are FP32
// on the vector units with a fixed summation order.
#include "rfm_internal.h"

#include <cmath>

namespace rfm {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f2bf(float x) {  // round to nearest, ties to even
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// C[m][n] = epi(sum_k A[m][k] B(n, k) + bias[n]) for m < M, n < N.
//   epi: act 1 -> tanh;  Hm != null -> times (1 - Hm[m][n]^2)
// BF16 path: B is bf16 [N rows][ldb] with ldb a multiple of 32 and zero padding past K.
// Workgroup: 4 wavefronts, 64 rows (16 per wavefront) x 64 columns (four 16-column tiles).
__global__ void __launch_bounds__(256) k_mlp_gemm_bf16(const float* __restrict__ A, int lda, int M, int K,
                                                       const uint16_t* __restrict__ B, int ldb, int N,
                                                       const float* __restrict__ bias, const float* __restrict__ Hm,
                                                       int ldh, int act, float* __restrict__ C, int ldc) {
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int q = lane / 16, c16 = lane % 16;
  const int m0 = blockIdx.x * 64 + wv * 16, n0 = blockIdx.y * 64;
  const int mr = m0 + c16;  // A row of this lane
  v4f acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = v4f{0, 0, 0, 0};
  for (int k0 = 0; k0 < ldb; k0 += 32) {
    uint16_t ab[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int k = k0 + 8 * q + j;
      ab[j] = (mr < M && k < K) ? f2bf(A[(int64_t)mr * lda + k]) : (uint16_t)0;
    }
    v8bf a;
    __builtin_memcpy(&a, ab, 16);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int n = n0 + 16 * t + c16;
      v8bf b = v8bf{};
      if (n < N) b = *reinterpret_cast<const v8bf*>(B + (int64_t)n * ldb + k0 + 8 * q);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
  }
  // lane (q, c) holds rows 4q + i, column c of each tile
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int n = n0 + 16 * t + c16;
    if (n >= N) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int m = m0 + 4 * q + i;
      if (m >= M) continue;
      float v = acc[t][i] + (bias ? bias[n] : 0.0f);
      if (act) v = tanhf(v);
      if (Hm) {
        const float h = Hm[(int64_t)m * ldh + n];
        v *= 1.0f - h * h;
      }
      C[(int64_t)m * ldc + n] = v;
    }
  }
}

// FP32 reference-precision form of the same product: B(n, k) = Bf[n * sn + k * sk]
__global__ void __launch_bounds__(256) k_mlp_gemm_f32(const float* __restrict__ A, int lda, int M, int K,
                                                      const float* __restrict__ Bf, int64_t sn, int64_t sk, int N,
                                                      const float* __restrict__ bias, const float* __restrict__ Hm,
                                                      int ldh, int act, float* __restrict__ C, int ldc) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)M * N) return;
  const int m = (int)(idx / N), n = (int)(idx % N);
  float s = 0.0f;
  for (int k = 0; k < K; ++k) s = fmaf(A[(int64_t)m * lda + k], Bf[n * sn + k * sk], s);
  float v = s + (bias ? bias[n] : 0.0f);
  if (act) v = tanhf(v);
  if (Hm) {
    const float h = Hm[(int64_t)m * ldh + n];
    v *= 1.0f - h * h;
  }
  C[(int64_t)m * ldc + n] = v;
}

// gW[n][k] = sum_m D[m][n] H[m][k],  gb[n] = sum_m D[m][n]  (16 x 16 output tile per workgroup,
// the batch in chunks of 64 rows through LDS; each output summed by one thread in row order)
__global__ void __launch_bounds__(256) k_mlp_wgrad(const float* __restrict__ Dl, int ldd, const float* __restrict__ H,
                                                   int ldh, int M, int N, int K, float* __restrict__ gW,
                                                   float* __restrict__ gb) {
  __shared__ float sd[64][17];
  __shared__ float sh[64][17];
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  const int n0 = blockIdx.y * 16, k0 = blockIdx.x * 16;
  const int n = n0 + ty, k = k0 + tx;
  float acc = 0.0f, accb = 0.0f;
  for (int mb = 0; mb < M; mb += 64) {
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int r = e / 16, c = e % 16;
      const int m = mb + r;
      sd[r][c] = (m < M && n0 + c < N) ? Dl[(int64_t)m * ldd + n0 + c] : 0.0f;
      sh[r][c] = (m < M && k0 + c < K) ? H[(int64_t)m * ldh + k0 + c] : 0.0f;
    }
    __syncthreads();
#pragma unroll 8
    for (int r = 0; r < 64; ++r) {
      acc = fmaf(sd[r][ty], sh[r][tx], acc);
      accb += sd[r][ty];
    }
    __syncthreads();
  }
  if (n < N && k < K) gW[(int64_t)n * K + k] = acc;
  if (gb && blockIdx.x == 0 && tx == 0 && n < N) gb[n] = accb;
}

// D[i] = 2 (Yp[i] - Y[i]) / count; partial sums of (Yp - Y)^2 per block (fixed order)
__global__ void __launch_bounds__(256) k_mlp_loss(const float* __restrict__ Yp, const float* __restrict__ Y,
                                                  int64_t cnt, float* __restrict__ D, double* __restrict__ part) {
  __shared__ double sh[256];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (i < cnt) {
    const float d = Yp[i] - Y[i];
    D[i] = 2.0f * d / (float)cnt;
    e = (double)d * d;
  }
  sh[threadIdx.x] = e;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Adam (Kingma & Ba, Algorithm 1): m, v moments, bias-corrected step
__global__ void k_adam(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ g, int64_t n, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / c1, vh = vi / c2;
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// BF16 copies of W [dout][din]: Wb [dout][Kp] and Wt [din][Np] (zero padding)
__global__ void k_mlp_cast(const float* __restrict__ W, int dout, int din, uint16_t* __restrict__ Wb, int Kp,
                           uint16_t* __restrict__ Wt, int Np) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nb = (int64_t)dout * Kp, nt = (int64_t)din * Np;
  if (i < nb) {
    const int r = (int)(i / Kp), c = (int)(i % Kp);
    Wb[i] = c < din ? f2bf(W[(int64_t)r * din + c]) : (uint16_t)0;
  }
  if (i < nt) {
    const int r = (int)(i / Np), c = (int)(i % Np);
    Wt[i] = c < dout ? f2bf(W[(int64_t)c * din + r]) : (uint16_t)0;
  }
}

// batch gather: rows idx[i] of X [n][dx], Y [n][dy]; idx from Philox4x64-10 (counter (step, i, 2, 0),
// key (seed, 0)), word 0 modulo n -- or the identity when the batch covers the data
__global__ void k_mlp_gather(const float* __restrict__ X, int dx, const float* __restrict__ Y, int dy, int64_t n,
                             int64_t bs, uint64_t seed, uint64_t step, float* __restrict__ Xb, float* __restrict__ Yb) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= bs) return;
  int64_t r = i;
  if (bs < n) {
    uint64_t c0 = step, c1 = (uint64_t)i, c2 = 2, c3 = 0, k0 = seed, k1 = 0;
    for (int rnd = 0; rnd < 10; ++rnd) {
      if (rnd) {
        k0 += 0x9E3779B97F4A7C15ull;
        k1 += 0xBB67AE8584CAA73Bull;
      }
      const uint64_t hi0 = __umul64hi(0xD2E7470EE14C6C93ull, c0), lo0 = 0xD2E7470EE14C6C93ull * c0;
      const uint64_t hi1 = __umul64hi(0xCA5A826395121157ull, c2), lo1 = 0xCA5A826395121157ull * c2;
      const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
      c0 = n0;
      c1 = lo1;
      c2 = n2;
      c3 = lo0;
    }
    r = (int64_t)(c0 % (uint64_t)n);
  }
  for (int j = 0; j < dx; ++j) Xb[i * dx + j] = X[r * dx + j];
  for (int j = 0; j < dy; ++j) Yb[i * dy + j] = Y[r * dy + j];
}

int pad32(int k) { return (k + 31) / 32 * 32; }

}  // namespace

struct Mlp {
  int in_dim = 0, width = 0, depth = 0, out_dim = 0, device = 0;
  hipStream_t stream = nullptr;
  int prec = RFM_PREC_BF16;
  int nl = 0;
  std::vector<int> din, dout, kp, np;
  std::vector<int64_t> woff, boff, wboff, wtoff;
  int64_t nparams = 0, nbf = 0, nbt = 0;
  DBuf<float> p, mom1, mom2, g;
  DBuf<uint16_t> wb, wt;
  DBuf<float> act, dlt, xb, yb, yd, xs, ys;
  DBuf<double> part;
  int64_t act_rows = 0;
  int64_t t = 0;  // Adam steps taken

  void alloc_rows(int64_t M) {
    if (M <= act_rows) return;
    int64_t tot = 0;
    for (int l = 0; l <= nl; ++l) tot += M * (l == 0 ? in_dim : (l == nl ? out_dim : width));
    act.resize((size_t)tot);
    dlt.resize((size_t)M * std::max(width, out_dim) * 2);
    yd.resize((size_t)M * out_dim);
    part.resize((size_t)((M * out_dim + 255) / 256 + 1));
    act_rows = M;
  }
  float* h(int l, int64_t M) {  // activation l ([M][dim_l]) inside act
    int64_t off = 0;
    for (int j = 0; j < l; ++j) off += M * (j == 0 ? in_dim : width);
    return act.p + off;
  }
  int hdim(int l) const { return l == 0 ? in_dim : (l == nl ? out_dim : width); }

  void recast() {
    for (int l = 0; l < nl; ++l) {
      const int64_t cnt = std::max<int64_t>((int64_t)dout[l] * kp[l], (int64_t)din[l] * np[l]);
      hipLaunchKernelGGL(k_mlp_cast, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, p.p + woff[l],
                         dout[l], din[l], wb.p + wboff[l], kp[l], wt.p + wtoff[l], np[l]);
    }
    RFM_HIP(hipGetLastError());
  }

  // C = epi(A B^T + bias) with B = W_l (transpose = false) or W_l^T (transpose = true)
  void gemm(int l, bool transpose, const float* A, int M, const float* bias, const float* Hm, int act_fn, float* C) {
    const int K = transpose ? dout[l] : din[l];
    const int N = transpose ? din[l] : dout[l];
    if (M == 0) return;
    if (prec == RFM_PREC_BF16) {
      const uint16_t* B = transpose ? wt.p + wtoff[l] : wb.p + wboff[l];
      const int ldb = transpose ? np[l] : kp[l];
      dim3 grid((unsigned)((M + 63) / 64), (unsigned)((N + 63) / 64));
      hipLaunchKernelGGL(k_mlp_gemm_bf16, grid, dim3(256), 0, stream, A, K, M, K, B, ldb, N, bias, Hm, N, act_fn, C,
                         N);
    } else {
      const float* W = p.p + woff[l];
      const int64_t sn = transpose ? 1 : din[l], sk = transpose ? din[l] : 1;
      const int64_t cnt = (int64_t)M * N;
      hipLaunchKernelGGL(k_mlp_gemm_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, stream, A, K, M, K, W, sn,
                         sk, N, bias, Hm, N, act_fn, C, N);
    }
    RFM_HIP(hipGetLastError());
  }

  // forward on device input X [M][in_dim] (copied into activation 0); returns the output pointer
  float* forward(const float* X, int64_t M) {
    alloc_rows(M);
    RFM_HIP(hipMemcpyAsync(h(0, M), X, (size_t)M * in_dim * 4, hipMemcpyDeviceToDevice, stream));
    for (int l = 0; l < nl; ++l)
      gemm(l, false, h(l, M), (int)M, p.p + boff[l], nullptr, l + 1 < nl ? 1 : 0, h(l + 1, M));
    return h(nl, M);
  }

  // MSE loss of the current batch and its gradient into g; returns the loss
  double loss_grad(const float* X, const float* Y, int64_t M) {
    float* out = forward(X, M);
    const int64_t cnt = M * out_dim;
    const int nb = (int)((cnt + 255) / 256);
    hipLaunchKernelGGL(k_mlp_loss, dim3(nb), dim3(256), 0, stream, out, Y, cnt, yd.p, part.p);
    RFM_HIP(hipGetLastError());
    // backward: delta of layer l's pre-activation is in cur [M][dout[l]]
    float* cur = yd.p;
    float* buf[2] = {dlt.p, dlt.p + (size_t)M * std::max(width, out_dim)};
    int which = 0;
    for (int l = nl - 1; l >= 0; --l) {
      const dim3 grid((unsigned)((din[l] + 15) / 16), (unsigned)((dout[l] + 15) / 16));
      hipLaunchKernelGGL(k_mlp_wgrad, grid, dim3(256), 0, stream, cur, dout[l], h(l, M), din[l], (int)M, dout[l],
                         din[l], g.p + woff[l], g.p + boff[l]);
      RFM_HIP(hipGetLastError());
      if (l > 0) {
        float* nxt = buf[which];
        which ^= 1;
        gemm(l, true, cur, (int)M, nullptr, h(l, M), 0, nxt);  // (delta W_l) * (1 - h_l^2)
        cur = nxt;
      }
    }
    std::vector<double> ph(nb);
    RFM_HIP(hipMemcpyAsync(ph.data(), part.p, nb * 8, hipMemcpyDeviceToHost, stream));
    RFM_HIP(hipStreamSynchronize(stream));
    double s = 0.0;
    for (double v : ph) s += v;
    return s / (double)cnt;
  }

  void adam(float lr, float b1, float b2, float eps) {
    ++t;
    const float c1 = 1.0f - std::pow(b1, (float)t), c2 = 1.0f - std::pow(b2, (float)t);
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((nparams + 255) / 256)), dim3(256), 0, stream, p.p, mom1.p, mom2.p, g.p,
                       nparams, lr, b1, b2, eps, c1, c2);
    RFM_HIP(hipGetLastError());
    recast();
  }
};

void mlp_check_shape(rfm_mlp* net, int in_dim, int out_dim) {
  RFM_CHECK(net != nullptr, RFM_EINVAL, "null network");
  const Mlp& M = *reinterpret_cast<const Mlp*>(net);
  RFM_CHECK(M.in_dim == in_dim && M.out_dim == out_dim, RFM_EINVAL,
            "network shape does not match (parameters + dim) -> ncomp");
}

}  // namespace rfm

using namespace rfm;

namespace {

Mlp& mget(rfm_mlp* h) {
  RFM_CHECK(h != nullptr, RFM_EINVAL, "null network");
  Mlp& M = *reinterpret_cast<Mlp*>(h);
  RFM_HIP(hipSetDevice(M.device));
  return M;
}

// host or device float array -> device buffer
void to_device(Mlp& M, DBuf<float>& dst, const float* src, size_t cnt) {
  dst.resize(std::max<size_t>(cnt, 1));
  if (cnt) RFM_HIP(hipMemcpyAsync(dst.p, src, cnt * 4, hipMemcpyDefault, M.stream));
}

}  // namespace

extern "C" {

rfm_status rfm_mlp_create(rfm_mlp** out, int32_t in_dim, int32_t width, int32_t depth, int32_t out_dim,
                          uint64_t seed, int32_t device, void* hip_stream) {
  return guarded([&] {
    RFM_CHECK(out != nullptr, RFM_EINVAL, "rfm_mlp_create: out is NULL");
    *out = nullptr;
    RFM_CHECK(in_dim >= 1 && in_dim <= 64 && out_dim >= 1 && out_dim <= 64, RFM_EINVAL,
              "rfm_mlp_create: in_dim and out_dim must be 1..64");
    RFM_CHECK(width >= 1 && width <= 1024 && depth >= 1 && depth <= 16, RFM_EINVAL,
              "rfm_mlp_create: width 1..1024, depth 1..16");
    int ndev = 0;
    RFM_HIP(hipGetDeviceCount(&ndev));
    RFM_CHECK(device >= 0 && device < ndev, RFM_EINVAL, "rfm_mlp_create: no such device");
    RFM_HIP(hipSetDevice(device));
    auto* M = new Mlp();
    std::unique_ptr<Mlp> guard(M);
    M->in_dim = in_dim;
    M->width = width;
    M->depth = depth;
    M->out_dim = out_dim;
    M->device = device;
    M->stream = reinterpret_cast<hipStream_t>(hip_stream);
    M->nl = depth + 1;
    int64_t off = 0, ob = 0, ot = 0;
    for (int l = 0; l < M->nl; ++l) {
      const int di = l == 0 ? in_dim : width, dn = l == depth ? out_dim : width;
      M->din.push_back(di);
      M->dout.push_back(dn);
      M->kp.push_back(pad32(di));
      M->np.push_back(pad32(dn));
      M->woff.push_back(off);
      off += (int64_t)dn * di;
      M->boff.push_back(off);
      off += dn;
      M->wboff.push_back(ob);
      ob += (int64_t)dn * pad32(di);
      M->wtoff.push_back(ot);
      ot += (int64_t)di * pad32(dn);
    }
    M->nparams = off;
    M->nbf = ob;
    M->nbt = ot;
    // Glorot-uniform weights from a seeded host generator (64-bit LCG, Knuth MMIX constants), zero biases
    std::vector<float> h(off, 0.0f);
    uint64_t st = seed * 0x9E3779B97F4A7C15ull + 1;
    for (int l = 0; l < M->nl; ++l) {
      const double lim = std::sqrt(6.0 / (M->din[l] + M->dout[l]));
      for (int64_t i = 0; i < (int64_t)M->dout[l] * M->din[l]; ++i) {
        st = st * 6364136223846793005ull + 1442695040888963407ull;
        const double u = (double)(st >> 11) * 0x1p-53;
        h[M->woff[l] + i] = (float)((2.0 * u - 1.0) * lim);
      }
    }
    M->p.resize(off);
    M->mom1.resize(off);
    M->mom2.resize(off);
    M->g.resize(off);
    M->wb.resize(ob);
    M->wt.resize(ot);
    RFM_HIP(hipMemcpyAsync(M->p.p, h.data(), off * 4, hipMemcpyHostToDevice, M->stream));
    RFM_HIP(hipMemsetAsync(M->mom1.p, 0, off * 4, M->stream));
    RFM_HIP(hipMemsetAsync(M->mom2.p, 0, off * 4, M->stream));
    M->recast();
    RFM_HIP(hipStreamSynchronize(M->stream));
    *out = reinterpret_cast<rfm_mlp*>(guard.release());
  });
}

void rfm_mlp_destroy(rfm_mlp* h) {
  if (!h) return;
  Mlp* M = reinterpret_cast<Mlp*>(h);
  (void)hipSetDevice(M->device);
  (void)hipStreamSynchronize(M->stream);
  delete M;
}

int64_t rfm_mlp_num_params(const rfm_mlp* h) { return h ? reinterpret_cast<const Mlp*>(h)->nparams : -1; }

rfm_status rfm_mlp_get_params(rfm_mlp* h, float* out) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(out != nullptr, RFM_EINVAL, "NULL argument");
    RFM_HIP(hipMemcpyAsync(out, M.p.p, M.nparams * 4, hipMemcpyDefault, M.stream));
    RFM_HIP(hipStreamSynchronize(M.stream));
  });
}

rfm_status rfm_mlp_set_params(rfm_mlp* h, const float* in) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(in != nullptr, RFM_EINVAL, "NULL argument");
    RFM_HIP(hipMemcpyAsync(M.p.p, in, M.nparams * 4, hipMemcpyDefault, M.stream));
    RFM_HIP(hipMemsetAsync(M.mom1.p, 0, M.nparams * 4, M.stream));
    RFM_HIP(hipMemsetAsync(M.mom2.p, 0, M.nparams * 4, M.stream));
    M.t = 0;
    M.recast();
    RFM_HIP(hipStreamSynchronize(M.stream));
  });
}

rfm_status rfm_mlp_set_precision(rfm_mlp* h, int32_t prec) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(prec == RFM_PREC_BF16 || prec == RFM_PREC_F32, RFM_EINVAL, "network precision must be BF16 or F32");
    M.prec = prec;
  });
}

rfm_status rfm_mlp_predict(rfm_mlp* h, const float* X, int64_t n, float* Y) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(n >= 0 && n < (int64_t)INT32_MAX, RFM_EINVAL, "rfm_mlp_predict: bad point count");
    RFM_CHECK((X && Y) || n == 0, RFM_EINVAL, "NULL argument");
    if (n == 0) return;
    to_device(M, M.xs, X, (size_t)n * M.in_dim);
    float* out = M.forward(M.xs.p, n);
    RFM_HIP(hipMemcpyAsync(Y, out, (size_t)n * M.out_dim * 4, hipMemcpyDefault, M.stream));
    RFM_HIP(hipStreamSynchronize(M.stream));
  });
}

rfm_status rfm_mlp_loss_grad(rfm_mlp* h, const float* X, const float* Y, int64_t n, double* loss, float* grad) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(n >= 1 && n < (int64_t)INT32_MAX, RFM_EINVAL, "rfm_mlp_loss_grad: bad sample count");
    RFM_CHECK(X && Y, RFM_EINVAL, "NULL argument");
    to_device(M, M.xs, X, (size_t)n * M.in_dim);
    to_device(M, M.ys, Y, (size_t)n * M.out_dim);
    const double L = M.loss_grad(M.xs.p, M.ys.p, n);
    if (loss) *loss = L;
    if (grad) {
      RFM_HIP(hipMemcpyAsync(grad, M.g.p, M.nparams * 4, hipMemcpyDefault, M.stream));
      RFM_HIP(hipStreamSynchronize(M.stream));
    }
  });
}

void rfm_train_opts_default(rfm_train_opts* o) {
  if (!o) return;
  o->steps = 2000;
  o->batch = 8192;
  o->lr = 1e-3f;
  o->beta1 = 0.9f;
  o->beta2 = 0.999f;
  o->eps = 1e-8f;
  o->lr_final = 0.0f;
  o->seed = 1;
}

rfm_status rfm_mlp_train(rfm_mlp* h, const float* X, const float* Y, int64_t n, const rfm_train_opts* o,
                         double* loss_log) {
  return guarded([&] {
    Mlp& M = mget(h);
    RFM_CHECK(o != nullptr, RFM_EINVAL, "rfm_mlp_train: opts is NULL");
    RFM_CHECK(n >= 1 && n < (int64_t)INT32_MAX, RFM_EINVAL, "rfm_mlp_train: bad sample count");
    RFM_CHECK(X && Y, RFM_EINVAL, "NULL argument");
    RFM_CHECK(o->steps >= 0 && o->batch >= 1, RFM_EINVAL, "rfm_mlp_train: bad steps or batch");
    RFM_CHECK(o->lr > 0 && o->lr_final >= 0 && o->beta1 >= 0 && o->beta1 < 1 && o->beta2 >= 0 && o->beta2 < 1 &&
                  o->eps > 0,
              RFM_EINVAL,
              "rfm_mlp_train: bad Adam settings");
    to_device(M, M.xs, X, (size_t)n * M.in_dim);
    to_device(M, M.ys, Y, (size_t)n * M.out_dim);
    const int64_t bs = std::min<int64_t>(o->batch, n);
    M.xb.resize((size_t)bs * M.in_dim);
    M.yb.resize((size_t)bs * M.out_dim);
    for (int s = 0; s < o->steps; ++s) {
      hipLaunchKernelGGL(k_mlp_gather, dim3((unsigned)((bs + 255) / 256)), dim3(256), 0, M.stream, M.xs.p, M.in_dim,
                         M.ys.p, M.out_dim, n, bs, o->seed, (uint64_t)s, M.xb.p, M.yb.p);
      RFM_HIP(hipGetLastError());
      const double L = M.loss_grad(M.xb.p, M.yb.p, bs);
      if (loss_log) loss_log[s] = L;
      float lr = o->lr;
      if (o->lr_final > 0 && o->steps > 1)
        lr = (float)(o->lr * std::pow((double)o->lr_final / o->lr, (double)s / (o->steps - 1)));
      M.adam(lr, o->beta1, o->beta2, o->eps);
    }
    RFM_HIP(hipStreamSynchronize(M.stream));
  });
}

}  // extern "C"
