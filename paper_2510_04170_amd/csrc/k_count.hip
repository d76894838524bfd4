// Count sketch B = S (D J) (the sketch of Sec. 4.1 as the paper uses it).
//
// S has one non-zero per column: S[h(r)][r] = sigma(r), with h(r) = word 0 mod s
// and sigma(r) = +1 if bit 0 of word 1 is clear (else -1) of Philox4x64-10 at
// counter (r, 0, 2, 0), key (seed, jac_index).  B costs one pass over the stored
// Jacobian: row r of D J, signed, is added to row h(r) of B.
//
// Determinism without atomics: on the host, the rows that touch each column
// block are grouped by bucket (sorted by bucket, then row); each group ("run")
// is summed in that fixed order by one wavefront, its lanes over the block's J
// columns, and written once.  Runs are kept in bucket order, so any range of
// B's rows is a contiguous range of runs: the streamed QR asks for B a block of
// rows at a time, and each block is cleared and then filled by its own runs.
#include <algorithm>
#include <chrono>

#include "rfm_internal.h"

namespace rfm {

namespace {

struct RunDesc {
  int32_t blk;     // column block
  int32_t bucket;  // row of B
  int32_t e0, e1;  // entries [e0, e1) of the run
};

// rows r0 .. r0 + nr - 1 of B (bucket b to out[c ldo + b - r0]) from runs [0, nruns) of that range
__global__ void __launch_bounds__(256) k_count_sketch(const RunDesc* __restrict__ runs, int64_t nruns,
                                                      const int64_t* __restrict__ eoff,
                                                      const double* __restrict__ esign,
                                                      const double* __restrict__ Jv, int J, int64_t r0, int64_t ldo,
                                                      double* __restrict__ out) {
  const int64_t k = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
  if (k >= nruns) return;
  const int lane = threadIdx.x % 64;
  const RunDesc rd = runs[k];
  double* bcol = out + (int64_t)rd.blk * J * ldo + (rd.bucket - r0);
  for (int c = lane; c < J; c += 64) {
    double acc = 0.0;
    for (int e = rd.e0; e < rd.e1; ++e) acc += esign[e] * Jv[eoff[e] + c];
    bcol[(int64_t)c * ldo] = acc;
  }
}

// out[c ldo + i] = 0 for i < nr, c < n
__global__ void k_zero_rows(double* __restrict__ out, int64_t ldo, int64_t nr, int64_t n) {
  const int64_t tot = nr * n;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < tot; q += st) {
    const int64_t c = q / nr, i = q - c * nr;
    out[c * ldo + i] = 0.0;
  }
}

__global__ void k_zero(double* __restrict__ x, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t st = (int64_t)gridDim.x * blockDim.x;
  for (int64_t j = i; j < n; j += st) x[j] = 0.0;
}

// Philox4x64-10 (Salmon et al., SC'11) on the host
void philox4x64_host(uint64_t c[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  for (int rnd = 0; rnd < 10; ++rnd) {
    if (rnd) {
      k0 += 0x9E3779B97F4A7C15ull;
      k1 += 0xBB67AE8584CAA73Bull;
    }
    const unsigned __int128 p0 = (unsigned __int128)M0 * c[0];
    const unsigned __int128 p1 = (unsigned __int128)M1 * c[2];
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

}  // namespace

void count_sketch_hash(int64_t r, int64_t s, uint64_t seed, uint64_t jac, int64_t* h, double* sigma) {
  uint64_t c[4] = {(uint64_t)r, 0, 2, 0};
  philox4x64_host(c, seed, jac);
  *h = (int64_t)(c[0] % (uint64_t)s);
  *sigma = (c[1] & 1ull) ? -1.0 : 1.0;
}

void prepare_count_sketch(Problem& P, uint64_t seed, uint64_t jac_index) {
  const int64_t s = P.s;
  const int nblk = P.geom.nbox * P.ncomp;
  RFM_CHECK(s >= 1 && s < (int64_t)INT32_MAX, RFM_EINVAL, "count sketch: sketch size out of range");
  // hash of every row
  std::vector<int64_t> h(P.m);
  std::vector<double> sg(P.m);
  for (int64_t r = 0; r < P.m; ++r) count_sketch_hash(r, s, seed, jac_index, &h[r], &sg[r]);
  // per column block: (bucket, row) pairs of the rows touching it, in order; runs of equal buckets
  std::vector<int64_t> eoff;
  std::vector<double> esign;
  std::vector<RunDesc> runs;
  std::vector<std::pair<int64_t, int64_t>> key;  // (bucket, entry offset in d_J)
  for (int bk = 0; bk < nblk; ++bk) {
    key.clear();
    for (int64_t sl = P.cbs_ptr_h[bk]; sl < P.cbs_ptr_h[bk + 1]; ++sl) {
      const int32_t g = P.slot_group_h[sl];
      if (g < 0) continue;
      for (int k = 0; k < 32; ++k) {
        const int64_t off = P.slot_rowoff_h[sl * 32 + k];
        if (off < 0) continue;
        const int64_t r = (int64_t)g * 32 + k;
        key.push_back({h[r] * P.m + r, off});
      }
    }
    std::sort(key.begin(), key.end());
    for (size_t i = 0; i < key.size();) {
      const int64_t b = key[i].first / P.m;
      RunDesc rd{bk, (int32_t)b, (int32_t)eoff.size(), 0};
      while (i < key.size() && key[i].first / P.m == b) {
        const int64_t r = key[i].first % P.m;
        eoff.push_back(key[i].second);
        esign.push_back(sg[r]);
        ++i;
      }
      rd.e1 = (int32_t)eoff.size();
      runs.push_back(rd);
    }
  }
  RFM_CHECK(eoff.size() < (size_t)INT32_MAX, RFM_EINVAL, "count sketch: too many entries");
  // bucket order (each run writes its own entries of B, so the order changes no value)
  std::stable_sort(runs.begin(), runs.end(), [](const RunDesc& a, const RunDesc& b) { return a.bucket < b.bucket; });
  P.cs_run_bucket.resize(runs.size());
  for (size_t k = 0; k < runs.size(); ++k) P.cs_run_bucket[k] = runs[k].bucket;
  DBuf<int64_t>& d_eoff = P.d_cs_eoff;
  DBuf<double>& d_esign = P.d_cs_sign;
  DBuf<char>& d_runs = P.d_cs_runs;
  d_eoff.resize(std::max<size_t>(1, eoff.size()));
  d_esign.resize(std::max<size_t>(1, esign.size()));
  d_runs.resize(std::max<size_t>(1, runs.size() * sizeof(RunDesc)));
  if (!eoff.empty()) {
    RFM_HIP(hipMemcpyAsync(d_eoff.p, eoff.data(), eoff.size() * 8, hipMemcpyHostToDevice, P.stream));
    RFM_HIP(hipMemcpyAsync(d_esign.p, esign.data(), esign.size() * 8, hipMemcpyHostToDevice, P.stream));
    RFM_HIP(hipMemcpyAsync(d_runs.p, runs.data(), runs.size() * sizeof(RunDesc), hipMemcpyHostToDevice, P.stream));
  }
  // the host vectors above must outlive the asynchronous copies
  RFM_HIP(hipStreamSynchronize(P.stream));
}

void launch_count_sketch_rows(Problem& P, int64_t r0, int64_t nr, double* out, int64_t ldo) {
  RFM_CHECK(r0 >= 0 && nr >= 0 && r0 + nr <= P.s && ldo >= nr, RFM_EINVAL, "count sketch: row range out of range");
  const auto lo = std::lower_bound(P.cs_run_bucket.begin(), P.cs_run_bucket.end(), (int32_t)r0);
  const auto hi = std::lower_bound(P.cs_run_bucket.begin(), P.cs_run_bucket.end(), (int32_t)(r0 + nr));
  const int64_t k0 = lo - P.cs_run_bucket.begin(), nruns = hi - lo;
  // algorithmic work: one signed add per stored Jacobian value (this range's share of them); bytes: those
  // values read once and written once into their buckets, the block cleared once
  const double share = (double)P.nvals * (double)nr / (double)P.s;
  ProfScope ps(P.prof, P.stream, "sketch_count", share, 8.0 * (2.0 * share + (double)nr * P.n));
  hipLaunchKernelGGL(k_zero_rows, dim3(4096), dim3(256), 0, P.stream, out, ldo, nr, P.n);
  if (nruns)
    hipLaunchKernelGGL(k_count_sketch, dim3((unsigned)((nruns + 3) / 4)), dim3(256), 0, P.stream,
                       reinterpret_cast<const RunDesc*>(P.d_cs_runs.p) + k0, nruns, P.d_cs_eoff.p, P.d_cs_sign.p,
                       P.d_J.p, P.J, r0, ldo, out);
  RFM_HIP(hipGetLastError());
}

void launch_count_sketch(Problem& P, uint64_t seed, uint64_t jac_index) {
  prepare_count_sketch(P, seed, jac_index);
  P.d_B.resize((size_t)P.s * P.n);
  launch_count_sketch_rows(P, 0, P.s, P.d_B.p, P.s);
}

double streamed_count_sketch_qr(Problem& P, uint64_t seed, uint64_t jac_index, int64_t rows_per_pass) {
  const auto t0 = std::chrono::steady_clock::now();
  prepare_count_sketch(P, seed, jac_index);
  const double t_prep = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  auto rows = [&](int64_t r0, int64_t nr, double* out, int64_t ldo) { launch_count_sketch_rows(P, r0, nr, out, ldo); };
  return t_prep + qr_factor_streamed(P, rows, qr_stream_rows(P, rows_per_pass));
}

}  // namespace rfm
