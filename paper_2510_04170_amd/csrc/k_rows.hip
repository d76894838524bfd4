// Row kernels: Jacobian/residual assembly with the row scale fused in, the
// directional products of the line search, phi(alpha), field evaluation and the
// block-sparse products J x and J^T y.
//
// One 64-wide wavefront owns one Jacobian row: lanes walk the row's features
// (feature j on lane j mod 64), so every value of the row is produced and
// written by consecutive lanes and the row's reductions (field values, the
// maximum for the scale, the dot products) are wavefront reductions.
#include <mutex>

#include "rfm_internal.h"

namespace rfm {

namespace {

constexpr int kWave = 64;
constexpr int kRowsPerBlock = 4;  // 256 threads, one row per wavefront

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ __forceinline__ double ipow(double x, int p) {
  double r = 1.0;
  for (int i = 0; i < p; ++i) r *= x;
  return r;
}

struct RowsCtx {
  GeomDesc g;
  const OpDesc* op;  // device copy: run-time indexing into an argument makes a private copy of it
  FeatDev f;
  const RowDesc* rows;
  const double* px;
  const double* pn;
  const double* rowdata;
};

// l_e(x) = (x - mu_e) / sigma_e, with the box bounds computed as lo + i h, + h
__device__ __forceinline__ void norm_coords(const GeomDesc& g, int e, const double* x, double* l) {
  int rem = e;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    if (a < g.dim) {
      int i = rem % g.nsub[a];
      rem /= g.nsub[a];
      double h = (g.hi[a] - g.lo[a]) / g.nsub[a];
      double blo = g.lo[a] + i * h;
      double bhi = blo + h;
      double mu = 0.5 * (blo + bhi);
      double sig = 0.5 * (bhi - blo);
      l[a] = (x[a] - mu) / sig;
    } else {
      l[a] = 0.0;
    }
  }
}

// t = tanh(k . l + b) of feature f
__device__ __forceinline__ double feat_t(const RowsCtx& C, int64_t f, const double* l) {
  double z = 0.0;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a)
    if (a < C.g.dim) z += C.f.W[a][f] * l[a];
  return tanh(z + C.f.b[f]);
}

// derivative selector applied to feature f with t = tanh(z)
__device__ __forceinline__ double feat_deriv(const RowsCtx& C, int deriv, int64_t f, double t) {
  double dt = 1.0 - t * t;
  if (deriv == RFM_D_ID) return t;
  if (deriv >= RFM_D_X0 && deriv <= RFM_D_X3) {
    // the weight table by an unrolled select (no run-time index into the argument)
    const double* ws = C.f.WS[0];
#pragma unroll
    for (int a = 1; a < kMaxDim; ++a)
      if (deriv - RFM_D_X0 == a) ws = C.f.WS[a];
    return dt * ws[f];
  }
  if (deriv == RFM_D_LAPLACE) return -2.0 * t * dt * C.f.S2[f];
  return -2.0 * t * dt * C.f.S2s[f];  // RFM_D_LAPLACE_SPACE
}

__device__ __forceinline__ double feat_normal(const RowsCtx& C, int64_t f, double t, const double* nrm) {
  double dt = 1.0 - t * t;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a)
    if (a < C.g.dim) s += C.f.WS[a][f] * nrm[a];
  return dt * s;
}

// Nonlinear part of PDE equation q at field values val[]: the sum of its
// polynomial and pointwise terms in Fp, and d Fp / d val[c] in dp[c].
__device__ __forceinline__ void nonlinear_terms(const RowsCtx& C, int q, const double* val, double& Fp,
                                                double* dp) {
  const int K = C.g.ncomp;
  Fp = 0.0;
#pragma unroll
  for (int c = 0; c < kMaxComp; ++c) dp[c] = 0.0;
  for (int i = 0; i < C.op->npoly; ++i) {
    if (C.op->poly_eq[i] != q) continue;
    double prod = C.op->poly_coeff[i];
    for (int c = 0; c < K; ++c) prod *= ipow(val[c], C.op->poly_pow[i][c]);
    Fp += prod;
    for (int c = 0; c < K; ++c) {
      const int pc = C.op->poly_pow[i][c];
      if (pc == 0) continue;
      double d = C.op->poly_coeff[i] * pc * ipow(val[c], pc - 1);
      for (int c2 = 0; c2 < K; ++c2)
        if (c2 != c) d *= ipow(val[c2], C.op->poly_pow[i][c2]);
      dp[c] += d;
    }
  }
  for (int i = 0; i < C.op->nfn; ++i) {
    if (C.op->fn_eq[i] != q) continue;
    const int c = C.op->fn_comp[i];
    double f, df;
    fn_eval(C.op->fn_kind[i], val[c], &f, &df);
    Fp += C.op->fn_coeff[i] * f;
    dp[c] += C.op->fn_coeff[i] * df;
  }
}

// v[q] for a run-time q < kMaxQ without dynamic register indexing
__device__ __forceinline__ double qsel(const double* v, int q) {
  double r = 0.0;
#pragma unroll
  for (int k = 0; k < kMaxQ; ++k)
    if (k == q) r = v[k];
  return r;
}

// Product terms coeff prod_k v_{q_k}^{p_k} of equation qrow at the field quantities vq[]: their sum
// added to Fp, and by the product rule d/dv_q of the sum added to dq[q].
__device__ __forceinline__ void prod_terms(const RowsCtx& C, int qrow, const double* vq, double& Fp, double* dq) {
  for (int i = 0; i < C.op->nprod; ++i) {
    if (C.op->prod_eq[i] != qrow) continue;
    const int nf = C.op->prod_nfac[i];
    const double coeff = C.op->prod_coeff[i];
    double fv[kMaxFac], fd[kMaxFac];
    double term = coeff;
#pragma unroll
    for (int k = 0; k < kMaxFac; ++k) {
      fv[k] = 1.0;
      fd[k] = 0.0;
      if (k < nf) {
        const double v = qsel(vq, C.op->prod_q[i][k]);
        const int pw = C.op->prod_pow[i][k];
        fv[k] = ipow(v, pw);
        fd[k] = pw * ipow(v, pw - 1);
        term *= fv[k];
      }
    }
    Fp += term;
#pragma unroll
    for (int k = 0; k < kMaxFac; ++k) {
      if (k >= nf) continue;
      double d = coeff * fd[k];
#pragma unroll
      for (int k2 = 0; k2 < kMaxFac; ++k2)
        if (k2 != k) d *= fv[k2];
      const int qk = C.op->prod_q[i][k];
#pragma unroll
      for (int qq = 0; qq < kMaxQ; ++qq)
        if (qq == qk) dq[qq] += d;
    }
  }
}

// sum over the field quantities q of component c of w[q] D_q phi_f (t = tanh of feature f)
__device__ __forceinline__ double quantity_comb(const RowsCtx& C, int c, int64_t f, double t, const double* w) {
  double r = 0.0;
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq)
    if (qq < C.op->nq && C.op->q_comp[qq] == c) r += w[qq] * feat_deriv(C, C.op->q_deriv[qq], f, t);
  return r;
}

// acc[q] += D_q phi_f * x for the field quantities q of component c
__device__ __forceinline__ void quantity_acc(const RowsCtx& C, int c, int64_t f, double t, double x, double* acc) {
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq)
    if (qq < C.op->nq && C.op->q_comp[qq] == c) acc[qq] += feat_deriv(C, C.op->q_deriv[qq], f, t) * x;
}

// Values of row r (positions c*J + j for PDE rows, j and J + j for continuity
// rows) in vals[], lane-strided; the unscaled residual (data included) in F.
// vals index: seg * KPER + k for feature j = lane + 64 k of segment/component seg.
template <int KPER>
__device__ __forceinline__ void row_values(const RowsCtx& C, int64_t r, const double* __restrict__ u, int lane,
                           double (&vals)[4 * KPER], double& F) {
  const RowDesc rd = C.rows[r];
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  double x[kMaxDim], l[kMaxDim], nrm[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    x[a] = a < dim ? C.px[(int64_t)rd.pt * dim + a] : 0.0;
    nrm[a] = a < dim ? C.pn[(int64_t)rd.pt * dim + a] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < 4 * KPER; ++i) vals[i] = 0.0;
  if (rd.kind == RFM_PDE) {
    const int q = rd.sel;
    norm_coords(C.g, rd.owner, x, l);
    double tv[4 * KPER];
    double accv[kMaxComp] = {0, 0, 0, 0};
    double accq[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    double accL = 0.0;
    const bool has_q = C.op->nq > 0;
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= K) break;
      const int64_t fb = ((int64_t)rd.owner * K + c) * J;
#pragma unroll
      for (int k = 0; k < KPER; ++k) {
        const int j = lane + kWave * k;
        tv[c * KPER + k] = 0.0;
        if (j < J) {
          const int64_t f = fb + j;
          const double t = feat_t(C, f, l);
          double Lv = 0.0;
          for (int i = 0; i < C.op->nlin; ++i)
            if (C.op->lin_eq[i] == q && C.op->lin_comp[i] == c) Lv += C.op->lin_coeff[i] * feat_deriv(C, C.op->lin_deriv[i], f, t);
          const double uj = u[f];
          accv[c] += t * uj;
          accL += Lv * uj;
          if (has_q) quantity_acc(C, c, f, t, uj, accq);
          vals[c * KPER + k] = Lv;
          tv[c * KPER + k] = t;
        }
      }
    }
    double val[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) val[c] = c < K ? wave_sum(accv[c]) : 0.0;
    accL = wave_sum(accL);
    double Fp, dp[kMaxComp];
    nonlinear_terms(C, q, val, Fp, dp);
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) {
      if (c >= K) break;
#pragma unroll
      for (int k = 0; k < KPER; ++k) vals[c * KPER + k] += dp[c] * tv[c * KPER + k];
    }
    if (has_q) {
      double vq[kMaxQ], dq[kMaxQ];
#pragma unroll
      for (int qq = 0; qq < kMaxQ; ++qq) {
        vq[qq] = qq < C.op->nq ? wave_sum(accq[qq]) : 0.0;
        dq[qq] = 0.0;
      }
      prod_terms(C, q, vq, Fp, dq);
#pragma unroll
      for (int c = 0; c < kMaxComp; ++c) {
        if (c >= K) break;
        const int64_t fb = ((int64_t)rd.owner * K + c) * J;
#pragma unroll
        for (int k = 0; k < KPER; ++k) {
          const int j = lane + kWave * k;
          if (j < J) vals[c * KPER + k] += quantity_comb(C, c, fb + j, tv[c * KPER + k], dq);
        }
      }
    }
    F = accL + Fp - C.rowdata[r];
  } else if (rd.kind == RFM_CONTINUITY) {
    const int c = rd.sel;
    double acc = 0.0;
#pragma unroll
    for (int seg = 0; seg < 2; ++seg) {
      const int e = seg == 0 ? rd.owner : rd.neighbor;
      norm_coords(C.g, e, x, l);
      const int64_t fb = ((int64_t)e * K + c) * J;
#pragma unroll
      for (int k = 0; k < KPER; ++k) {
        const int j = lane + kWave * k;
        if (j < J) {
          const int64_t f = fb + j;
          const double t = feat_t(C, f, l);
          double v = rd.order == 0 ? t : feat_normal(C, f, t, nrm);
          if (seg) v = -v;
          vals[seg * KPER + k] = v;
          acc += v * u[f];
        }
      }
    }
    F = wave_sum(acc);
  } else {  // Dirichlet or Neumann
    const int c = rd.sel;
    norm_coords(C.g, rd.owner, x, l);
    const int64_t fb = ((int64_t)rd.owner * K + c) * J;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < KPER; ++k) {
      const int j = lane + kWave * k;
      if (j < J) {
        const int64_t f = fb + j;
        const double t = feat_t(C, f, l);
        const double v = rd.kind == RFM_DIRICHLET ? t : feat_normal(C, f, t, nrm);
        vals[k] = v;
        acc += v * u[f];
      }
    }
    F = wave_sum(acc) - C.rowdata[r];
  }
}

// store position of vals[idx] in the row, or -1
template <int KPER>
__device__ __forceinline__ int val_pos(int kind, int J, int idx, int lane) {
  const int seg = idx / KPER, k = idx % KPER;
  const int j = lane + kWave * k;
  if (j >= J) return -1;
  if (kind == RFM_PDE) return seg * J + j;
  if (kind == RFM_CONTINUITY) return seg < 2 ? seg * J + j : -1;
  return seg == 0 ? j : -1;
}

template <int KPER>
__global__ void __launch_bounds__(256) k_assemble(RowsCtx C, const TileDesc* __restrict__ tiles,
                                                  const int32_t* __restrict__ rowtile, int64_t m,
                                                  const double* __restrict__ u, double cscale,
                                                  double* __restrict__ Jv, double* __restrict__ DF,
                                                  double* __restrict__ Dout) {
  const int lane = threadIdx.x % kWave;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= m) return;
  double vals[4 * KPER];
  double F;
  row_values<KPER>(C, r, u, lane, vals, F);
  const int kind = C.rows[r].kind;
  double mx = 0.0;
#pragma unroll
  for (int i = 0; i < 4 * KPER; ++i) mx = fmax(mx, fabs(vals[i]));
  mx = wave_max(mx);
  const double D = mx > 0.0 ? cscale / mx : 1.0;
  const TileDesc td = tiles[rowtile[r]];
  const int w = td.wA + td.wB;
  double* row = Jv + td.val_off + (int64_t)(r - td.row0) * w;
#pragma unroll
  for (int i = 0; i < 4 * KPER; ++i) {
    const int pos = val_pos<KPER>(kind, C.g.J, i, lane);
    if (pos >= 0 && pos < w) row[pos] = D * vals[i];
  }
  if (lane == 0) {
    DF[r] = D * F;
    Dout[r] = D;
  }
}

// Rows wider than the register-held form (more than 512 features per box):
// the row is swept three times, recomputing every feature value each time
// (tanh is cheap next to the row's store): the field values and the linear
// part for the residual and the nonlinear derivatives, then the row maximum
// for the scale, then the scaled values into the stored row.  Entry (seg, j):
// segment seg is the component of a PDE row or the side of a continuity row.
__device__ __forceinline__ double wide_entry(const RowsCtx& C, const RowDesc& rd, const double* l,
                                             const double* nrm, int64_t f, int seg, double& t) {
  t = feat_t(C, f, l);
  if (rd.kind == RFM_PDE) {
    double Lv = 0.0;
    for (int i = 0; i < C.op->nlin; ++i)
      if (C.op->lin_eq[i] == rd.sel && C.op->lin_comp[i] == seg)
        Lv += C.op->lin_coeff[i] * feat_deriv(C, C.op->lin_deriv[i], f, t);
    return Lv;
  }
  double v;
  if (rd.kind == RFM_CONTINUITY) {
    v = rd.order == 0 ? t : feat_normal(C, f, t, nrm);
    return seg ? -v : v;
  }
  return rd.kind == RFM_DIRICHLET ? t : feat_normal(C, f, t, nrm);
}

__global__ void __launch_bounds__(256) k_assemble_wide(RowsCtx C, const TileDesc* __restrict__ tiles,
                                                       const int32_t* __restrict__ rowtile, int64_t m,
                                                       const double* __restrict__ u, double cscale,
                                                       double* __restrict__ Jv, double* __restrict__ DF,
                                                       double* __restrict__ Dout) {
  const int lane = threadIdx.x % kWave;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= m) return;
  const RowDesc rd = C.rows[r];
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  double x[kMaxDim], nrm[kMaxDim], l[2][kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    x[a] = a < dim ? C.px[(int64_t)rd.pt * dim + a] : 0.0;
    nrm[a] = a < dim ? C.pn[(int64_t)rd.pt * dim + a] : 0.0;
  }
  norm_coords(C.g, rd.owner, x, l[0]);
  const bool cont = rd.kind == RFM_CONTINUITY;
  if (cont) norm_coords(C.g, rd.neighbor, x, l[1]);
  const int nseg = rd.kind == RFM_PDE ? K : (cont ? 2 : 1);
  // feature block of segment seg
  auto fbase = [&](int seg) -> int64_t {
    if (rd.kind == RFM_PDE) return ((int64_t)rd.owner * K + seg) * J;
    const int e = (cont && seg) ? rd.neighbor : rd.owner;
    return ((int64_t)e * K + rd.sel) * J;
  };
  // sweep 1: sums
  double accv[kMaxComp] = {0, 0, 0, 0};
  double accq[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  double accL = 0.0;
  const bool has_q = rd.kind == RFM_PDE && C.op->nq > 0;
  for (int seg = 0; seg < nseg; ++seg) {
    const int64_t fb = fbase(seg);
    const double* ls = l[cont ? seg : 0];
    double av = 0.0;
    for (int j = lane; j < J; j += kWave) {
      double t;
      const double v = wide_entry(C, rd, ls, nrm, fb + j, seg, t);
      const double uj = u[fb + j];
      accL += v * uj;
      av += t * uj;
      if (has_q) quantity_acc(C, seg, fb + j, t, uj, accq);
    }
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c == seg) accv[c] = av;
  }
  accL = wave_sum(accL);
  double dp[kMaxComp] = {0, 0, 0, 0};
  double dq[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  double F;
  if (rd.kind == RFM_PDE) {
    double val[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) val[c] = c < K ? wave_sum(accv[c]) : 0.0;
    double Fp;
    nonlinear_terms(C, rd.sel, val, Fp, dp);
    if (has_q) {
      double vq[kMaxQ];
#pragma unroll
      for (int qq = 0; qq < kMaxQ; ++qq) vq[qq] = qq < C.op->nq ? wave_sum(accq[qq]) : 0.0;
      prod_terms(C, rd.sel, vq, Fp, dq);
    }
    F = accL + Fp - C.rowdata[r];
  } else {
    F = accL - (cont ? 0.0 : C.rowdata[r]);
  }
  // sweep 2: row maximum
  double mx = 0.0;
  for (int seg = 0; seg < nseg; ++seg) {
    const int64_t fb = fbase(seg);
    const double* ls = l[cont ? seg : 0];
    double dps = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c == seg) dps = dp[c];
    for (int j = lane; j < J; j += kWave) {
      double t;
      const double v = wide_entry(C, rd, ls, nrm, fb + j, seg, t);
      const double w = has_q ? quantity_comb(C, seg, fb + j, t, dq) : 0.0;
      mx = fmax(mx, fabs(v + dps * t + w));
    }
  }
  mx = wave_max(mx);
  const double D = mx > 0.0 ? cscale / mx : 1.0;
  // sweep 3: scaled values
  const TileDesc td = tiles[rowtile[r]];
  const int w = td.wA + td.wB;
  double* row = Jv + td.val_off + (int64_t)(r - td.row0) * w;
  for (int seg = 0; seg < nseg; ++seg) {
    const int64_t fb = fbase(seg);
    const double* ls = l[cont ? seg : 0];
    double dps = 0.0;
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c)
      if (c == seg) dps = dp[c];
    for (int j = lane; j < J; j += kWave) {
      double t;
      const double v = wide_entry(C, rd, ls, nrm, fb + j, seg, t);
      const double wq = has_q ? quantity_comb(C, seg, fb + j, t, dq) : 0.0;
      const int pos = seg * J + j;
      if (pos < w) row[pos] = D * (v + dps * t + wq);
    }
  }
  if (lane == 0) {
    DF[r] = D * F;
    Dout[r] = D;
  }
}

// ---------------------------------------------------------------------------
// smooth partition of unity: psi_e(x) = prod_a b(l_a(x)) with b = 1 on |y| <= 3/4,
// (1 - sin(2 pi |y|)) / 2 on 3/4 <= |y| <= 5/4, 0 beyond, and b = 1 on the side of an axis where
// the box touches the boundary of the domain.  A row's boxes are its tile's segments.
// ---------------------------------------------------------------------------

struct Pou {
  double psi, g[kMaxDim], h, hs;  // value, gradient, sum of pure second derivatives (all axes; space)
  double l[kMaxDim];              // the box's local coordinates of the point
};

__device__ __forceinline__ Pou pou_smooth(const GeomDesc& G, int e, const double* x) {
  Pou P;
  double f[kMaxDim], d1[kMaxDim], d2[kMaxDim];
  int rem = e;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    f[a] = 1.0;
    d1[a] = 0.0;
    d2[a] = 0.0;
    P.l[a] = 0.0;
    if (a < G.dim) {
      const int i = rem % G.nsub[a];
      rem /= G.nsub[a];
      const double hw = (G.hi[a] - G.lo[a]) / G.nsub[a];
      const double blo = G.lo[a] + i * hw, bhi = blo + hw;
      const double mu = 0.5 * (blo + bhi), sig = 0.5 * (bhi - blo);
      const double y = (x[a] - mu) / sig, ay = fabs(y);
      P.l[a] = y;
      const bool flat = (i == 0 && y < 0.0) || (i == G.nsub[a] - 1 && y > 0.0);
      if (!flat && ay > 0.75) {
        if (ay < 1.25) {
          double sn, cs;
          sincospi(2.0 * ay, &sn, &cs);
          f[a] = 0.5 * (1.0 - sn);
          d1[a] = -M_PI * cs * (y < 0.0 ? -1.0 : 1.0) / sig;
          d2[a] = 2.0 * M_PI * M_PI * sn / (sig * sig);
        } else {
          f[a] = 0.0;
        }
      }
    }
  }
  P.psi = 1.0;
  P.h = 0.0;
  P.hs = 0.0;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) P.psi *= f[a];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    double o = 1.0;
#pragma unroll
    for (int b2 = 0; b2 < kMaxDim; ++b2)
      if (b2 != a) o *= f[b2];
    P.g[a] = d1[a] * o;
    P.h += d2[a] * o;
    if (a < G.dim - 1) P.hs += d2[a] * o;
  }
  return P;
}

// the weight table of axis a (an unrolled select: no run-time index into the argument)
__device__ __forceinline__ const double* ws_of(const RowsCtx& C, int a) {
  const double* ws = C.f.WS[0];
#pragma unroll
  for (int k = 1; k < kMaxDim; ++k)
    if (a == k) ws = C.f.WS[k];
  return ws;
}

// derivative selector applied to psi phi_f (t = tanh of feature f) by the product rule
__device__ __forceinline__ double smooth_deriv(const RowsCtx& C, int deriv, int64_t f, double t, const Pou& P) {
  const double dt = 1.0 - t * t;
  if (deriv == RFM_D_ID) return P.psi * t;
  if (deriv >= RFM_D_X0 && deriv <= RFM_D_X3) {
    const int a = deriv - RFM_D_X0;
    double ga = 0.0;
#pragma unroll
    for (int k = 0; k < kMaxDim; ++k)
      if (k == a) ga = P.g[k];
    return P.psi * dt * ws_of(C, a)[f] + t * ga;
  }
  const bool space = deriv == RFM_D_LAPLACE_SPACE;
  const int na = space ? C.g.dim - 1 : C.g.dim;
  double cross = 0.0;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a)
    if (a < na) cross += P.g[a] * C.f.WS[a][f];
  const double s2 = space ? C.f.S2s[f] : C.f.S2[f];
  return P.psi * (-2.0 * t * dt * s2) + 2.0 * dt * cross + t * (space ? P.hs : P.h);
}

__device__ __forceinline__ double smooth_normal(const RowsCtx& C, int64_t f, double t, const Pou& P,
                                                const double* nrm) {
  const double dt = 1.0 - t * t;
  double sw = 0.0, sg = 0.0;
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a)
    if (a < C.g.dim) {
      sw += C.f.WS[a][f] * nrm[a];
      sg += P.g[a] * nrm[a];
    }
  return P.psi * dt * sw + t * sg;
}

// one entry of a smooth-partition row without the nonlinear parts: the linear operator of equation q on
// component c (PDE rows), or the boundary operator
__device__ __forceinline__ double smooth_lin_entry(const RowsCtx& C, const RowDesc& rd, int c, int64_t f, double t,
                                                   const Pou& P, const double* nrm) {
  if (rd.kind == RFM_PDE) {
    double Lv = 0.0;
    for (int i = 0; i < C.op->nlin; ++i)
      if (C.op->lin_eq[i] == rd.sel && C.op->lin_comp[i] == c)
        Lv += C.op->lin_coeff[i] * smooth_deriv(C, C.op->lin_deriv[i], f, t, P);
    return Lv;
  }
  return rd.kind == RFM_DIRICHLET ? P.psi * t : smooth_normal(C, f, t, P, nrm);
}

__device__ __forceinline__ double smooth_quantity_comb(const RowsCtx& C, int c, int64_t f, double t, const Pou& P,
                                                       const double* w) {
  double r = 0.0;
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq)
    if (qq < C.op->nq && C.op->q_comp[qq] == c) r += w[qq] * smooth_deriv(C, C.op->q_deriv[qq], f, t, P);
  return r;
}

__device__ __forceinline__ void smooth_quantity_acc(const RowsCtx& C, int c, int64_t f, double t, const Pou& P,
                                                    double x, double* acc) {
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq)
    if (qq < C.op->nq && C.op->q_comp[qq] == c) acc[qq] += smooth_deriv(C, C.op->q_deriv[qq], f, t, P) * x;
}

// Rows of the smooth partition (PDE, Dirichlet, Neumann), swept three times like k_assemble_wide:
// sums, maximum, scaled store.  Segment sg of the tile is box seg_col[sg] / (K J); PDE rows hold all K
// components of each box (position sg wseg + c J + j), boundary rows component sel (sg wseg + j).
__global__ void __launch_bounds__(256) k_assemble_smooth(RowsCtx C, const TileDesc* __restrict__ tiles,
                                                         const int32_t* __restrict__ rowtile, int64_t m,
                                                         const double* __restrict__ u, double cscale,
                                                         double* __restrict__ Jv, double* __restrict__ DF,
                                                         double* __restrict__ Dout) {
  const int lane = threadIdx.x % kWave;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= m) return;
  const RowDesc rd = C.rows[r];
  const TileDesc td = tiles[rowtile[r]];
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  const bool pde = rd.kind == RFM_PDE;
  const int c0 = pde ? 0 : rd.sel, c1 = pde ? K : rd.sel + 1;
  double x[kMaxDim], nrm[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    x[a] = a < dim ? C.px[(int64_t)rd.pt * dim + a] : 0.0;
    nrm[a] = a < dim ? C.pn[(int64_t)rd.pt * dim + a] : 0.0;
  }
  const bool has_q = pde && C.op->nq > 0;
  // sweep 1: sums
  double accv[kMaxComp] = {0, 0, 0, 0};
  double accq[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  double accL = 0.0;
  for (int sg = 0; sg < td.nseg; ++sg) {
    const int e = td.seg_col[sg] / (K * J);
    const Pou P = pou_smooth(C.g, e, x);
    for (int c = c0; c < c1; ++c) {
      const int64_t fb = ((int64_t)e * K + c) * J;
      double av = 0.0;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        const double t = feat_t(C, f, P.l);
        const double uj = u[f];
        accL += smooth_lin_entry(C, rd, c, f, t, P, nrm) * uj;
        av += P.psi * t * uj;
        if (has_q) smooth_quantity_acc(C, c, f, t, P, uj, accq);
      }
#pragma unroll
      for (int k = 0; k < kMaxComp; ++k)
        if (k == c) accv[k] += av;
    }
  }
  accL = wave_sum(accL);
  double dp[kMaxComp] = {0, 0, 0, 0};
  double dq[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  double F;
  if (pde) {
    double val[kMaxComp];
#pragma unroll
    for (int c = 0; c < kMaxComp; ++c) val[c] = c < K ? wave_sum(accv[c]) : 0.0;
    double Fp;
    nonlinear_terms(C, rd.sel, val, Fp, dp);
    if (has_q) {
      double vq[kMaxQ];
#pragma unroll
      for (int qq = 0; qq < kMaxQ; ++qq) vq[qq] = qq < C.op->nq ? wave_sum(accq[qq]) : 0.0;
      prod_terms(C, rd.sel, vq, Fp, dq);
    }
    F = accL + Fp - C.rowdata[r];
  } else {
    F = accL - C.rowdata[r];
  }
  // the value of entry (box of segment sg, component c, feature f)
  auto entry = [&](const Pou& P, int c, int64_t f, double t) -> double {
    double v = smooth_lin_entry(C, rd, c, f, t, P, nrm);
    if (pde) {
      double dpc = 0.0;
#pragma unroll
      for (int k = 0; k < kMaxComp; ++k)
        if (k == c) dpc = dp[k];
      v += dpc * P.psi * t;
      if (has_q) v += smooth_quantity_comb(C, c, f, t, P, dq);
    }
    return v;
  };
  // sweep 2: row maximum
  double mx = 0.0;
  for (int sg = 0; sg < td.nseg; ++sg) {
    const int e = td.seg_col[sg] / (K * J);
    const Pou P = pou_smooth(C.g, e, x);
    for (int c = c0; c < c1; ++c) {
      const int64_t fb = ((int64_t)e * K + c) * J;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        mx = fmax(mx, fabs(entry(P, c, f, feat_t(C, f, P.l))));
      }
    }
  }
  mx = wave_max(mx);
  const double D = mx > 0.0 ? cscale / mx : 1.0;
  // sweep 3: scaled values
  double* row = Jv + td.val_off + (int64_t)(r - td.row0) * td.wA;
  for (int sg = 0; sg < td.nseg; ++sg) {
    const int e = td.seg_col[sg] / (K * J);
    const Pou P = pou_smooth(C.g, e, x);
    for (int c = c0; c < c1; ++c) {
      const int64_t fb = ((int64_t)e * K + c) * J;
      double* rs = row + sg * td.wseg + (c - c0) * J;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        rs[j] = D * entry(P, c, f, feat_t(C, f, P.l));
      }
    }
  }
  if (lane == 0) {
    DF[r] = D * F;
    Dout[r] = D;
  }
}

// the line search's per-row record (layout of k_row_eval) for smooth-partition rows
__global__ void __launch_bounds__(256) k_row_eval_smooth(RowsCtx C, const TileDesc* __restrict__ tiles,
                                                         const int32_t* __restrict__ rowtile, int64_t m,
                                                         const double* __restrict__ u,
                                                         const double* __restrict__ du, double* __restrict__ ab) {
  const int lane = threadIdx.x % kWave;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= m) return;
  const RowDesc rd = C.rows[r];
  const TileDesc td = tiles[rowtile[r]];
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  const int nq = C.op->nq;
  const int stride = 2 + 2 * K + 2 * nq;
  const bool pde = rd.kind == RFM_PDE;
  const int c0 = pde ? 0 : rd.sel, c1 = pde ? K : rd.sel + 1;
  double x[kMaxDim], nrm[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    x[a] = a < dim ? C.px[(int64_t)rd.pt * dim + a] : 0.0;
    nrm[a] = a < dim ? C.pn[(int64_t)rd.pt * dim + a] : 0.0;
  }
  double au = 0.0, ad = 0.0;
  double vu[kMaxComp] = {0, 0, 0, 0}, vd[kMaxComp] = {0, 0, 0, 0};
  double qu[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0}, qd[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int sg = 0; sg < td.nseg; ++sg) {
    const int e = td.seg_col[sg] / (K * J);
    const Pou P = pou_smooth(C.g, e, x);
    for (int c = c0; c < c1; ++c) {
      const int64_t fb = ((int64_t)e * K + c) * J;
      double su = 0.0, sd = 0.0;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        const double t = feat_t(C, f, P.l);
        const double a = u[f], d = du ? du[f] : 0.0;
        const double Lv = smooth_lin_entry(C, rd, c, f, t, P, nrm);
        au += Lv * a;
        ad += Lv * d;
        su += P.psi * t * a;
        sd += P.psi * t * d;
        if (pde && nq) {
          smooth_quantity_acc(C, c, f, t, P, a, qu);
          smooth_quantity_acc(C, c, f, t, P, d, qd);
        }
      }
#pragma unroll
      for (int k = 0; k < kMaxComp; ++k)
        if (k == c) {
          vu[k] += su;
          vd[k] += sd;
        }
    }
  }
  au = wave_sum(au);
  ad = wave_sum(ad);
  for (int c = 0; c < K; ++c) {
    vu[c] = wave_sum(vu[c]);
    vd[c] = wave_sum(vd[c]);
  }
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq)
    if (qq < nq) {
      qu[qq] = wave_sum(qu[qq]);
      qd[qq] = wave_sum(qd[qq]);
    }
  if (lane == 0) {
    double* o = ab + r * stride;
    o[0] = au - C.rowdata[r];
    o[1] = ad;
    for (int c = 0; c < K; ++c) {
      o[2 + c] = vu[c];
      o[2 + K + c] = vd[c];
    }
#pragma unroll
    for (int qq = 0; qq < kMaxQ; ++qq)
      if (qq < nq) {
        o[2 + 2 * K + qq] = qu[qq];
        o[2 + 2 * K + nq + qq] = qd[qq];
      }
  }
}

// u_n(x) (GRAD: its gradient, out [npts][ncomp][dim]) with the smooth partition: the owner's neighbours
// whose support holds x; d_a (psi phi) = psi d_a phi + phi d_a psi
template <bool GRAD>
__global__ void __launch_bounds__(256) k_eval_points_smooth(RowsCtx C, int64_t npts, const double* __restrict__ x,
                                                            const int32_t* __restrict__ owner,
                                                            const double* __restrict__ u, double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (p >= npts) return;
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  double xx[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) xx[a] = a < dim ? x[p * dim + a] : 0.0;
  int idx[kMaxDim];
  int rem = owner[p];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    idx[a] = a < dim ? rem % C.g.nsub[a] : 0;
    if (a < dim) rem /= C.g.nsub[a];
  }
  double acc[kMaxComp] = {0, 0, 0, 0};
  double accg[kMaxComp][kMaxDim] = {};
  int ncand = 1;
  for (int a = 0; a < dim; ++a) ncand *= 3;
  for (int k = 0; k < ncand; ++k) {
    int kk = k, e = 0, stride = 1;
    bool ok = true;
#pragma unroll
    for (int a = 0; a < kMaxDim; ++a) {
      if (a >= dim) continue;
      const int ia = idx[a] + kk % 3 - 1;
      kk /= 3;
      if (ia < 0 || ia >= C.g.nsub[a]) ok = false;
      e += ia * stride;
      stride *= C.g.nsub[a];
    }
    if (!ok) continue;
    const Pou P = pou_smooth(C.g, e, xx);
    if (P.psi == 0.0) continue;
    for (int c = 0; c < K; ++c) {
      const int64_t fb = ((int64_t)e * K + c) * J;
      double s = 0.0, sg[kMaxDim] = {};
      for (int j = lane; j < J; j += kWave) {
        const double t = feat_t(C, fb + j, P.l);
        s += t * u[fb + j];
        if (GRAD) {
          const double w = (1.0 - t * t) * u[fb + j];
#pragma unroll
          for (int a = 0; a < kMaxDim; ++a)
            if (a < dim) sg[a] += C.f.WS[a][fb + j] * w;
        }
      }
#pragma unroll
      for (int q = 0; q < kMaxComp; ++q)
        if (q == c) {
          acc[q] += P.psi * s;
          if (GRAD) {
#pragma unroll
            for (int a = 0; a < kMaxDim; ++a) accg[q][a] += P.psi * sg[a] + P.g[a] * s;
          }
        }
    }
  }
#pragma unroll
  for (int c = 0; c < kMaxComp; ++c) {
    if (c >= K) continue;
    if (GRAD) {
#pragma unroll
      for (int a = 0; a < kMaxDim; ++a) {
        if (a >= dim) continue;
        const double v = wave_sum(accg[c][a]);
        if (lane == 0) out[(p * K + c) * dim + a] = v;
      }
    } else {
      const double v = wave_sum(acc[c]);
      if (lane == 0) out[p * K + c] = v;
    }
  }
}

// Linear part and field values along u and du for the line search:
//   ab[r] = {a_r, b_r, vu_0..vu_{K-1}, vd_0..vd_{K-1}, qu_0..qu_{nq-1}, qd_0..qd_{nq-1}}
//   F_r(alpha) = a_r + alpha b_r + sum_poly coeff prod_c (vu_c + alpha vd_c)^p_c
//                + sum_fn coeff f(vu_c + alpha vd_c) + sum_prod coeff prod_k (qu_k + alpha qd_k)^p_k
// (qu, qd: the product terms' field quantities along u and du)
template <int KPER>
__global__ void __launch_bounds__(256) k_row_eval(RowsCtx C, int64_t m, const double* __restrict__ u,
                                                  const double* __restrict__ du, double* __restrict__ ab) {
  const int lane = threadIdx.x % kWave;
  const int64_t r = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (r >= m) return;
  const RowDesc rd = C.rows[r];
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  const int nq = C.op->nq;
  const int stride = 2 + 2 * K + 2 * nq;
  double x[kMaxDim], l[kMaxDim], nrm[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) {
    x[a] = a < dim ? C.px[(int64_t)rd.pt * dim + a] : 0.0;
    nrm[a] = a < dim ? C.pn[(int64_t)rd.pt * dim + a] : 0.0;
  }
  double au = 0.0, ad = 0.0;
  double vu[kMaxComp] = {0, 0, 0, 0}, vd[kMaxComp] = {0, 0, 0, 0};
  double qu[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0}, qd[kMaxQ] = {0, 0, 0, 0, 0, 0, 0, 0};
  if (rd.kind == RFM_PDE) {
    const int q = rd.sel;
    norm_coords(C.g, rd.owner, x, l);
    for (int c = 0; c < K; ++c) {
      const int64_t fb = ((int64_t)rd.owner * K + c) * J;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        const double t = feat_t(C, f, l);
        double Lv = 0.0;
        for (int i = 0; i < C.op->nlin; ++i)
          if (C.op->lin_eq[i] == q && C.op->lin_comp[i] == c) Lv += C.op->lin_coeff[i] * feat_deriv(C, C.op->lin_deriv[i], f, t);
        const double a = u[f];
        const double d = du ? du[f] : 0.0;
        vu[c] += t * a;
        vd[c] += t * d;
        au += Lv * a;
        ad += Lv * d;
        if (nq) {
          quantity_acc(C, c, f, t, a, qu);
          quantity_acc(C, c, f, t, d, qd);
        }
      }
    }
  } else if (rd.kind == RFM_CONTINUITY) {
    const int c = rd.sel;
    for (int seg = 0; seg < 2; ++seg) {
      const int e = seg == 0 ? rd.owner : rd.neighbor;
      norm_coords(C.g, e, x, l);
      const int64_t fb = ((int64_t)e * K + c) * J;
      for (int j = lane; j < J; j += kWave) {
        const int64_t f = fb + j;
        const double t = feat_t(C, f, l);
        double v = rd.order == 0 ? t : feat_normal(C, f, t, nrm);
        if (seg) v = -v;
        au += v * u[f];
        ad += du ? v * du[f] : 0.0;
      }
    }
  } else {
    const int c = rd.sel;
    norm_coords(C.g, rd.owner, x, l);
    const int64_t fb = ((int64_t)rd.owner * K + c) * J;
    for (int j = lane; j < J; j += kWave) {
      const int64_t f = fb + j;
      const double t = feat_t(C, f, l);
      const double v = rd.kind == RFM_DIRICHLET ? t : feat_normal(C, f, t, nrm);
      au += v * u[f];
      ad += du ? v * du[f] : 0.0;
    }
  }
  au = wave_sum(au);
  ad = wave_sum(ad);
  for (int c = 0; c < K; ++c) {
    vu[c] = wave_sum(vu[c]);
    vd[c] = wave_sum(vd[c]);
  }
#pragma unroll
  for (int qq = 0; qq < kMaxQ; ++qq) {
    if (qq < nq) {
      qu[qq] = wave_sum(qu[qq]);
      qd[qq] = wave_sum(qd[qq]);
    }
  }
  if (lane == 0) {
    double* o = ab + r * stride;
    o[0] = au - (rd.kind == RFM_CONTINUITY ? 0.0 : C.rowdata[r]);
    o[1] = ad;
    for (int c = 0; c < K; ++c) {
      o[2 + c] = vu[c];
      o[2 + K + c] = vd[c];
    }
#pragma unroll
    for (int qq = 0; qq < kMaxQ; ++qq) {
      if (qq < nq) {
        o[2 + 2 * K + qq] = qu[qq];
        o[2 + 2 * K + nq + qq] = qd[qq];
      }
    }
  }
}

constexpr int kRedBlock = 256;

// sum over rows of (D_r F_r(alpha))^2 -> one partial per block; optional F output
__global__ void __launch_bounds__(kRedBlock) k_phi(RowsCtx C, int64_t m, const double* __restrict__ ab,
                                                   double alpha, const double* __restrict__ D,
                                                   double* __restrict__ partial, double* __restrict__ Fout) {
  __shared__ double sh[kRedBlock];
  const int K = C.g.ncomp;
  const int nq = C.op->nq;
  const int stride = 2 + 2 * K + 2 * nq;
  double acc = 0.0;
  for (int64_t r = (int64_t)blockIdx.x * kRedBlock + threadIdx.x; r < m; r += (int64_t)gridDim.x * kRedBlock) {
    const double* o = ab + r * stride;
    double F = o[0] + alpha * o[1];
    const RowDesc rd = C.rows[r];
    if (rd.kind == RFM_PDE) {
      for (int i = 0; i < C.op->npoly; ++i) {
        if (C.op->poly_eq[i] != rd.sel) continue;
        double prod = C.op->poly_coeff[i];
        for (int c = 0; c < K; ++c) prod *= ipow(o[2 + c] + alpha * o[2 + K + c], C.op->poly_pow[i][c]);
        F += prod;
      }
      for (int i = 0; i < C.op->nfn; ++i) {
        if (C.op->fn_eq[i] != rd.sel) continue;
        const int c = C.op->fn_comp[i];
        double f, df;
        fn_eval(C.op->fn_kind[i], o[2 + c] + alpha * o[2 + K + c], &f, &df);
        F += C.op->fn_coeff[i] * f;
      }
      for (int i = 0; i < C.op->nprod; ++i) {
        if (C.op->prod_eq[i] != rd.sel) continue;
        double term = C.op->prod_coeff[i];
        for (int k = 0; k < C.op->prod_nfac[i]; ++k) {
          const int qk = C.op->prod_q[i][k];
          term *= ipow(o[2 + 2 * K + qk] + alpha * o[2 + 2 * K + nq + qk], C.op->prod_pow[i][k]);
        }
        F += term;
      }
    }
    if (Fout) Fout[r] = F;
    const double s = D ? D[r] * F : F;
    acc += s * s;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kRedBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

// fixed-order sum of nparts partials into out[0]
__global__ void __launch_bounds__(kRedBlock) k_reduce_sum(const double* __restrict__ partial, int nparts,
                                                          double* __restrict__ out) {
  __shared__ double sh[kRedBlock];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += kRedBlock) acc += partial[i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int h = kRedBlock / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) sh[threadIdx.x] += sh[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = sh[0];
}

// u_n(x) at arbitrary points, one wavefront per point (GRAD: the gradient, out [npts][ncomp][dim], from
// d_a phi = (1 - t^2) w_a / sigma_a)
template <bool GRAD>
__global__ void __launch_bounds__(256) k_eval_points(RowsCtx C, int64_t npts, const double* __restrict__ x,
                                                     const int32_t* __restrict__ owner,
                                                     const double* __restrict__ u, double* __restrict__ out) {
  const int lane = threadIdx.x % kWave;
  const int64_t p = (int64_t)blockIdx.x * kRowsPerBlock + threadIdx.x / kWave;
  if (p >= npts) return;
  const int K = C.g.ncomp, J = C.g.J, dim = C.g.dim;
  const int e = owner[p];
  double xx[kMaxDim], l[kMaxDim];
#pragma unroll
  for (int a = 0; a < kMaxDim; ++a) xx[a] = a < dim ? x[p * dim + a] : 0.0;
  norm_coords(C.g, e, xx, l);
  for (int c = 0; c < K; ++c) {
    const int64_t fb = ((int64_t)e * K + c) * J;
    if (GRAD) {
      double g[kMaxDim] = {};
      for (int j = lane; j < J; j += kWave) {
        const double t = feat_t(C, fb + j, l);
        const double w = (1.0 - t * t) * u[fb + j];
#pragma unroll
        for (int a = 0; a < kMaxDim; ++a)
          if (a < dim) g[a] += C.f.WS[a][fb + j] * w;
      }
#pragma unroll
      for (int a = 0; a < kMaxDim; ++a) {
        if (a >= dim) continue;
        const double v = wave_sum(g[a]);
        if (lane == 0) out[(p * K + c) * dim + a] = v;
      }
    } else {
      double acc = 0.0;
      for (int j = lane; j < J; j += kWave) acc += feat_t(C, fb + j, l) * u[fb + j];
      acc = wave_sum(acc);
      if (lane == 0) out[p * K + c] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// block-sparse products on the stored (scaled) Jacobian
// ---------------------------------------------------------------------------

// Block-sparse products, one 64-row tile per workgroup (four wavefronts).  A tile's values are one
// contiguous row-major block (nrows x w).  When w and the tile's offset are multiples of the 16-byte
// vector (4 FP32 or 2 FP64 values) and w <= 1024, every lane owns fixed 16-byte
// column slices of the row (vector k of lane l starts at value (64 k + l) VEC): it reads its slices
// of each row with one 16-byte load per slice, keeps the matching x values (J x) or partial column
// sums (J^T y) in registers across the tile's rows, and the cross-lane work is done once per tile
// through LDS.  Other tiles (odd widths, rows wider than the register budget) take the plain loops.
constexpr int kVecWidth = 1024;  // widest row on the vector path

template <typename T>
struct Vec16;
template <>
struct Vec16<float> {
  static constexpr int N = 4;
  static constexpr int K = kVecWidth / (64 * 4);  // 16-byte slices per lane and row
  __device__ static void load(const float* p, double* o) {
    const float4 v = *reinterpret_cast<const float4*>(p);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  }
};
template <>
struct Vec16<double> {
  static constexpr int N = 2;
  static constexpr int K = kVecWidth / (64 * 2);
  __device__ static void load(const double* p, double* o) {
    const double2 v = *reinterpret_cast<const double2*>(p);
    o[0] = v.x;
    o[1] = v.y;
  }
};

template <typename T>
__device__ __forceinline__ bool tile_vector_path(const TileDesc& td, int w) {
  constexpr int V = Vec16<T>::N;
  return w % V == 0 && td.val_off % V == 0 && w <= kVecWidth;
}

// y[r] = sum_p J[r,p] x[col(p)] - ucoef * uprev[r];  optional ||y||^2 partial per tile;
// ucoef = alpha/beta is read from the LSQR state when st != null.  Wavefront wv of the tile's
// workgroup takes rows wv, wv + 4, ...: every lane reads its 16-byte slices of those rows (the loads
// of all of them can be in flight together), and the row sums are wavefront reductions at the end.
template <typename T>
__global__ void __launch_bounds__(256) k_jmul(const TileDesc* __restrict__ tiles, const T* __restrict__ Jv,
                                              const double* __restrict__ x, double* __restrict__ y,
                                              const double* __restrict__ uprev, const LsqrState* __restrict__ st,
                                              double* __restrict__ partial) {
  if (st && st->done) return;
  constexpr int V = Vec16<T>::N, NK = Vec16<T>::K;
  constexpr int RPW = kTileRows / kRowsPerBlock;  // rows per wavefront
  __shared__ double sh[kRowsPerBlock];
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  const TileDesc td = tiles[blockIdx.x];
  const int w = td.wA + td.wB;
  const int32_t* seg_col = tiles[blockIdx.x].seg_col;  // run-time index: read from memory
  const double uc = st ? st->alpha * st->inv_beta : 0.0;  // x arrives already scaled by 1/alpha
  const T* tile = Jv + td.val_off;
  double acc[RPW];
#pragma unroll
  for (int j = 0; j < RPW; ++j) acc[j] = 0.0;
  if (tile_vector_path<T>(td, w)) {
    // this lane's x values: column slices k = 0 .. NK - 1
    double xv[NK][V];
#pragma unroll
    for (int k = 0; k < NK; ++k)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const int pos = (k * kWave + lane) * V + v;
        xv[k][v] = pos < w ? x[seg_col[pos / td.wseg] + pos % td.wseg] : 0.0;
      }
#pragma unroll
    for (int j = 0; j < RPW; ++j) {
      const int rr = wv + kRowsPerBlock * j;
      if (rr < td.nrows) {
        const T* row = tile + (int64_t)rr * w;
#pragma unroll
        for (int k = 0; k < NK; ++k) {
          const int pos = (k * kWave + lane) * V;
          if (pos < w) {
            double val[V];
            Vec16<T>::load(row + pos, val);
#pragma unroll
            for (int v = 0; v < V; ++v) acc[j] += val[v] * xv[k][v];
          }
        }
      }
    }
  } else {
    for (int j = 0; j < RPW; ++j) {
      const int rr = wv + kRowsPerBlock * j;
      if (rr < td.nrows) {
        const T* row = tile + (int64_t)rr * w;
        double a = 0.0;
        for (int sg = 0; sg < td.nseg; ++sg) {
          const T* rs = row + sg * td.wseg;
          const double* xs = x + seg_col[sg];
          for (int p = lane; p < td.wseg; p += kWave) a += (double)rs[p] * xs[p];
        }
        acc[j] = a;
      }
    }
  }
  double nrm = 0.0;
#pragma unroll
  for (int j = 0; j < RPW; ++j) {
    const int rr = wv + kRowsPerBlock * j;
    double v = wave_sum(acc[j]);
    if (rr < td.nrows) {
      const int64_t r = td.row0 + rr;
      if (uprev) v -= uc * uprev[r];
      if (lane == 0) y[r] = v;
      nrm += v * v;
    }
  }
  if (partial) {
    if (lane == 0) sh[wv] = nrm;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  }
}

// part[tile slot + p] = sum_{rows} J[r,p] y[r] * yscale.  nk wavefronts per tile, nk = the widest
// row's count of 64-lane 16-byte column slices, so that every slice of every tile has a wavefront of its
// own at any row width: on the vector path (width and offset multiples of the 16-byte vector) wavefront
// k sums slice k over the tile's rows, reading one 16-byte piece per row, with y of row r broadcast from
// lane r, and no cross-lane work; off it, wavefront k takes columns k * 64 + lane, stepping by nk * 64.
template <typename T>
__global__ void __launch_bounds__(kWave) k_jtmul_tiles(const TileDesc* __restrict__ tiles,
                                                       const T* __restrict__ Jv, const double* __restrict__ y,
                                                       const LsqrState* __restrict__ st, double* __restrict__ part,
                                                       int nk) {
  if (st && st->done) return;
  constexpr int V = Vec16<T>::N;
  const int t = blockIdx.x / nk, k = blockIdx.x % nk;
  const int lane = threadIdx.x;
  const TileDesc td = tiles[t];
  const int w = td.wA + td.wB;
  const double ysc = st ? st->inv_beta : 1.0;
  const T* tile = Jv + td.val_off;
  const double yl = lane < td.nrows ? y[td.row0 + lane] * ysc : 0.0;  // lane r holds row r's y
  if (w % V == 0 && td.val_off % V == 0) {
    const int pos = (k * kWave + lane) * V;
    if (k * kWave * V >= w) return;  // this slice lies past the row
    double acc[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
    const bool in = pos < w;
#pragma unroll 16
    for (int rr = 0; rr < td.nrows; ++rr) {
      const double yr = __shfl(yl, rr, kWave);
      if (in) {
        double val[V];
        Vec16<T>::load(tile + (int64_t)rr * w + pos, val);
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] += val[v] * yr;
      }
    }
    if (in) {
#pragma unroll
      for (int v = 0; v < V; ++v) part[td.part_off + pos + v] = acc[v];
    }
  } else {
    if (k * kWave >= w) return;  // uniform over the workgroup
    // lanes leave the column loop at different times: y goes through LDS, not through lane exchanges
    __shared__ double ys[kTileRows];
    ys[lane] = yl;
    __syncthreads();
    for (int p = k * kWave + lane; p < w; p += nk * kWave) {
      double acc = 0.0;
      const T* col = tile + p;
      for (int rr = 0; rr < td.nrows; ++rr) acc += (double)col[(int64_t)rr * w] * ys[rr];
      part[td.part_off + p] = acc;
    }
  }
}

// wavefronts per tile of k_jtmul_tiles: 16-byte column slices of 64 lanes in the widest row
template <typename T>
static int jtmul_slices(const Problem& P) {
  const int per = kWave * Vec16<T>::N;
  return std::max(1, (P.max_tile_w + per - 1) / per);
}

// x[j] = sum over the tiles touching column block j / J, in tile order
__global__ void __launch_bounds__(256) k_jtmul_reduce(const TileDesc* __restrict__ tiles,
                                                      const int32_t* __restrict__ cb_ptr,
                                                      const int32_t* __restrict__ cb_tile,
                                                      const int32_t* __restrict__ cb_off, int J, int64_t n,
                                                      const double* __restrict__ part, const LsqrState* __restrict__ st,
                                                      double* __restrict__ x) {
  if (st && st->done) return;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t blk = j / J;
  const int jj = (int)(j - blk * J);
  double acc = 0.0;
  for (int k = cb_ptr[blk]; k < cb_ptr[blk + 1]; ++k) acc += part[tiles[cb_tile[k]].part_off + cb_off[k] + jj];
  x[j] = acc;
}

// dense copy of rows [r0, r0 + nrows) of the stored Jacobian
__global__ void k_jac_rows(const TileDesc* __restrict__ tiles, const int32_t* __restrict__ rowtile,
                           const double* __restrict__ Jv, int64_t r0, int64_t nrows, int64_t n,
                           double* __restrict__ out) {
  const int64_t rr = blockIdx.x;
  if (rr >= nrows) return;
  const int64_t r = r0 + rr;
  const TileDesc td = tiles[rowtile[r]];
  const int w = td.wA + td.wB;
  double* o = out + rr * n;
  for (int64_t c = threadIdx.x; c < n; c += blockDim.x) o[c] = 0.0;
  __syncthreads();
  const double* row = Jv + td.val_off + (int64_t)(r - td.row0) * w;
  for (int p = threadIdx.x; p < w; p += blockDim.x) {
    const int col = td.seg_col[p / td.wseg] + p % td.wseg;
    o[col] = row[p];
  }
}

RowsCtx make_ctx(Problem& P) {
  RowsCtx C;
  C.g = P.geom;
  C.op = device_op(P);
  C.f = P.feat;
  C.rows = P.d_rows.p;
  C.px = P.d_px.p;
  C.pn = P.d_pnormal.p;
  C.rowdata = P.d_rowdata.p;
  return C;
}

int kper_of(const Problem& P) { return (P.J + kWave - 1) / kWave; }

}  // namespace

void launch_assemble(Problem& P, const double* u, double c) {
  ProfScope ps(P.prof, P.stream, "assemble", 0.0, 8.0 * ((double)P.nvals + 2.0 * P.m + P.n));
  RowsCtx C = make_ctx(P);
  dim3 grid((unsigned)((P.m + kRowsPerBlock - 1) / kRowsPerBlock));
  if (P.geom.pou == RFM_POU_SMOOTH) {
    hipLaunchKernelGGL(k_assemble_smooth, grid, dim3(256), 0, P.stream, C, P.d_tiles.p, P.d_rowtile.p, P.m, u, c,
                       P.d_J.p, P.d_DF.p, P.d_D.p);
    RFM_HIP(hipGetLastError());
    return;
  }
  switch (kper_of(P)) {
#define RFM_CASE(KP)                                                                                    \
  case KP:                                                                                              \
    hipLaunchKernelGGL(k_assemble<KP>, grid, dim3(256), 0, P.stream, C, P.d_tiles.p, P.d_rowtile.p, P.m, u, c, \
                       P.d_J.p, P.d_DF.p, P.d_D.p);                                                     \
    break;
    RFM_CASE(1) RFM_CASE(2) RFM_CASE(3) RFM_CASE(4) RFM_CASE(5) RFM_CASE(6) RFM_CASE(7) RFM_CASE(8)
#undef RFM_CASE
    default:
      hipLaunchKernelGGL(k_assemble_wide, grid, dim3(256), 0, P.stream, C, P.d_tiles.p, P.d_rowtile.p, P.m, u, c,
                         P.d_J.p, P.d_DF.p, P.d_D.p);
  }
  RFM_HIP(hipGetLastError());
}

void launch_row_eval(Problem& P, const double* u, const double* du, double* out_ab) {
  ProfScope ps(P.prof, P.stream, "linesearch_products", 0.0, 8.0 * ((double)P.m * (2 + 2 * P.ncomp) + 2.0 * P.n));
  RowsCtx C = make_ctx(P);
  dim3 grid((unsigned)((P.m + kRowsPerBlock - 1) / kRowsPerBlock));
  if (P.geom.pou == RFM_POU_SMOOTH)
    hipLaunchKernelGGL(k_row_eval_smooth, grid, dim3(256), 0, P.stream, C, P.d_tiles.p, P.d_rowtile.p, P.m, u, du,
                       out_ab);
  else
    hipLaunchKernelGGL(k_row_eval<1>, grid, dim3(256), 0, P.stream, C, P.m, u, du, out_ab);
  RFM_HIP(hipGetLastError());
}

int reduce_blocks_rows(const Problem& P) {
  int64_t b = (P.m + kRedBlock - 1) / kRedBlock;
  return (int)std::min<int64_t>(std::max<int64_t>(b, 1), 1024);
}

void launch_phi(Problem& P, const double* ab, double alpha, const double* D, double* out_sumsq) {
  ProfScope ps(P.prof, P.stream, "linesearch_phi", 0.0, 8.0 * (double)P.m * (3 + 2 * P.ncomp));
  RowsCtx C = make_ctx(P);
  const int nb = reduce_blocks_rows(P);
  hipLaunchKernelGGL(k_phi, dim3(nb), dim3(kRedBlock), 0, P.stream, C, P.m, ab, alpha, D, P.d_red.p, nullptr);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedBlock), 0, P.stream, P.d_red.p, nb, out_sumsq);
  RFM_HIP(hipGetLastError());
}

void launch_residual_from_ab(Problem& P, const double* ab, double* F, double* out_sumsq) {
  RowsCtx C = make_ctx(P);
  const int nb = reduce_blocks_rows(P);
  hipLaunchKernelGGL(k_phi, dim3(nb), dim3(kRedBlock), 0, P.stream, C, P.m, ab, 0.0, (const double*)nullptr,
                     P.d_red.p, F);
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedBlock), 0, P.stream, P.d_red.p, nb, out_sumsq);
  RFM_HIP(hipGetLastError());
}

void launch_reduce_sum(Problem& P, const double* partials, int nparts, double* out) {
  hipLaunchKernelGGL(k_reduce_sum, dim3(1), dim3(kRedBlock), 0, P.stream, partials, nparts, out);
  RFM_HIP(hipGetLastError());
}

void launch_eval_points(Problem& P, const double* u, int64_t npts, const double* x, const int32_t* owner,
                        double* out, bool grad) {
  if (npts == 0) return;
  RowsCtx C = make_ctx(P);
  dim3 grid((unsigned)((npts + kRowsPerBlock - 1) / kRowsPerBlock));
  if (P.geom.pou == RFM_POU_SMOOTH) {
    if (grad)
      hipLaunchKernelGGL(k_eval_points_smooth<true>, grid, dim3(256), 0, P.stream, C, npts, x, owner, u, out);
    else
      hipLaunchKernelGGL(k_eval_points_smooth<false>, grid, dim3(256), 0, P.stream, C, npts, x, owner, u, out);
  } else {
    if (grad)
      hipLaunchKernelGGL(k_eval_points<true>, grid, dim3(256), 0, P.stream, C, npts, x, owner, u, out);
    else
      hipLaunchKernelGGL(k_eval_points<false>, grid, dim3(256), 0, P.stream, C, npts, x, owner, u, out);
  }
  RFM_HIP(hipGetLastError());
}

template <typename T>
static void jmul_impl(Problem& P, const T* J, const double* x, double* y, const double* u_prev, const LsqrState* st,
                      double* red_partials) {
  ProfScope ps(P.prof, P.stream, sizeof(T) == 8 ? "jmul" : "jmul_f32", 2.0 * P.nvals,
               sizeof(T) * (double)P.nvals + 8.0 * (P.n + (u_prev ? 2.0 : 1.0) * P.m));
  hipLaunchKernelGGL(k_jmul<T>, dim3(P.ntiles), dim3(256), 0, P.stream, P.d_tiles.p, J, x, y, u_prev, st,
                     red_partials);
  RFM_HIP(hipGetLastError());
}

void launch_jmul(Problem& P, const double* J, const double* x, double* y, const double* u_prev,
                 const LsqrState* st, double* red_partials) {
  jmul_impl(P, J, x, y, u_prev, st, red_partials);
}

void launch_jmul(Problem& P, const float* J, const double* x, double* y, const double* u_prev, const LsqrState* st,
                 double* red_partials) {
  jmul_impl(P, J, x, y, u_prev, st, red_partials);
}

template <typename T>
static void jtmul_impl(Problem& P, const T* J, const double* y, double* x, const LsqrState* st) {
  ProfScope ps(P.prof, P.stream, sizeof(T) == 8 ? "jtmul" : "jtmul_f32", 2.0 * P.nvals,
               sizeof(T) * (double)P.nvals + 8.0 * (P.m + P.n));
  const int nk = jtmul_slices<T>(P);
  hipLaunchKernelGGL(k_jtmul_tiles<T>, dim3((unsigned)(P.ntiles * nk)), dim3(kWave), 0, P.stream, P.d_tiles.p, J, y,
                     st, P.d_part.p, nk);
  hipLaunchKernelGGL(k_jtmul_reduce, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, P.stream, P.d_tiles.p,
                     P.d_cb_ptr.p, P.d_cb_tile.p, P.d_cb_off.p, P.J, P.n, P.d_part.p, st, x);
  RFM_HIP(hipGetLastError());
}

void launch_jtmul(Problem& P, const double* J, const double* y, double* x, const LsqrState* st) {
  jtmul_impl(P, J, y, x, st);
}

void launch_jtmul(Problem& P, const float* J, const double* y, double* x, const LsqrState* st) {
  jtmul_impl(P, J, y, x, st);
}

// ---------------------------------------------------------------------------
// J^T y without allocation (rfm_jtmul_noalloc): the tile partials live in a fixed device array instead
// of the problem's buffer.  Every GPU the library runs on holds its own copy of the array (64 MiB) until
// the process ends; its device address is looked up once per device, with that device current, and
// only that address is handed to kernels (the array's name is a host-side stand-in).
// ---------------------------------------------------------------------------
constexpr int kMaxDevices = 64;
constexpr size_t kNoallocDoubles = (size_t)8 << 20;  // 64 MiB of partial sums
static __device__ __align__(256) double scratch[kNoallocDoubles];
static std::mutex g_scratch_mu;
static double* g_scratch[kMaxDevices] = {};

size_t noalloc_scratch_doubles() { return kNoallocDoubles; }

double* noalloc_scratch(int device) {
  RFM_CHECK(device >= 0 && device < kMaxDevices, RFM_EINVAL, "device index out of range for the fixed scratch");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[device]) {
    int cur = -1;
    RFM_HIP(hipGetDevice(&cur));
    RFM_CHECK(cur == device, RFM_EINVAL, "internal: the scratch is looked up with its device current");
    double* ptr = nullptr;
    RFM_HIP(hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)));
    RFM_CHECK(ptr != nullptr, RFM_EDEVICE, "no device address for the fixed scratch");
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}

void launch_jtmul_noalloc(Problem& P, const double* y, double* x, double* part) {
  const int nk = jtmul_slices<double>(P);
  hipLaunchKernelGGL(k_jtmul_tiles<double>, dim3((unsigned)(P.ntiles * nk)), dim3(kWave), 0, P.stream,
                     P.d_tiles.p, P.d_J.p, y, nullptr, part, nk);
  hipLaunchKernelGGL(k_jtmul_reduce, dim3((unsigned)((P.n + 255) / 256)), dim3(256), 0, P.stream, P.d_tiles.p,
                     P.d_cb_ptr.p, P.d_cb_tile.p, P.d_cb_off.p, P.J, P.n, part, nullptr, x);
  RFM_HIP(hipGetLastError());
}

void launch_jacobian_rows(Problem& P, int64_t r0, int64_t nrows, double* out) {
  hipLaunchKernelGGL(k_jac_rows, dim3((unsigned)nrows), dim3(256), 0, P.stream, P.d_tiles.p, P.d_rowtile.p, P.d_J.p,
                     r0, nrows, P.n, out);
  RFM_HIP(hipGetLastError());
}

}  // namespace rfm
