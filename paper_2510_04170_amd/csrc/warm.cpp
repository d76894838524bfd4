// Projection of field values onto the random-feature basis and the learned
// initial guess built on it.
//
// The fit min || D (Phi u - f) || uses the same machinery as a Newton step of
// the method (Alg. 1 steps 2-5) on the linear problem "u_n(x) = f(x) at the
// PDE points": assembly gives D Phi and D (Phi 0 - f), the sketch and QR give
// R (kept, since Phi does not change between calls), LSQR on D Phi R^-1 and
// one triangular solve give the coefficients.
#include <cmath>

#include "rfm_internal.h"

namespace rfm {

namespace {

Problem& problem_of(rfm_problem* h) { return *reinterpret_cast<Problem*>(h); }

void check(rfm_status rc) {
  if (rc != RFM_OK) throw Error(rc, rfm_last_error());
}

int64_t pde_points(const Problem& P) {
  int64_t k = 0;
  for (const auto& g : P.groups)
    if (g.kind == RFM_PDE) k += g.npts;
  return k;
}

// the identity-operator problem on the PDE points of P, with R formed
void build_projection(Problem& P, const rfm_solve_opts& o) {
  if (P.proj && P.proj_gamma == o.sketch_factor && P.proj_seed == o.sketch_seed && P.proj_c == o.row_scale_c) return;
  if (P.proj) {
    rfm_destroy(P.proj);
    P.proj = nullptr;
  }
  rfm_problem* h = nullptr;
  check(rfm_create(&h, P.dim, P.ncomp, P.device, P.stream));
  P.proj = h;
  int32_t nsub[kMaxDim];
  for (int a = 0; a < P.dim; ++a) nsub[a] = P.geom.nsub[a];
  check(rfm_set_partition(h, P.geom.lo, P.geom.hi, nsub));
  check(rfm_set_partition_of_unity(h, P.geom.pou));
  check(rfm_set_features(h, P.J, P.W.data(), P.b.data()));
  for (const auto& g : P.groups) {
    if (g.kind != RFM_PDE || g.npts == 0) continue;
    std::vector<double> zeros((size_t)g.npts * P.ncomp, 0.0);
    check(rfm_add_points(h, RFM_PDE, g.npts, P.px.data() + g.pt0 * P.dim, g.owner, -1, nullptr, -1, 1,
                         zeros.data()));
  }
  std::vector<rfm_lin_term> lin(P.ncomp);
  for (int c = 0; c < P.ncomp; ++c) lin[c] = rfm_lin_term{c, c, 1.0, RFM_D_ID};
  check(rfm_set_operator(h, lin.data(), P.ncomp, nullptr, 0));
  check(rfm_finalize(h));
  Problem& Q = problem_of(h);
  Q.d_u.resize(Q.n);
  RFM_HIP(hipMemsetAsync(Q.d_u.p, 0, Q.n * sizeof(double), Q.stream));
  launch_assemble(Q, Q.d_u.p, o.row_scale_c);
  Q.have_J = true;
  Q.cur_c = o.row_scale_c;
  Q.s = (int64_t)std::ceil(o.sketch_factor * (double)Q.n);
  launch_sketch(Q, o.sketch_seed, 0, RFM_PREC_F64);
  Q.have_B = true;
  qr_factor(Q);  // throws RFM_ESINGULAR
  Q.have_B = false;
  Q.have_R = true;
  RFM_HIP(hipStreamSynchronize(Q.stream));
  P.proj_gamma = o.sketch_factor;
  P.proj_seed = o.sketch_seed;
  P.proj_c = o.row_scale_c;
}

void project(Problem& P, const rfm_solve_opts& o, const double* values, double* u_out, double* resnorm) {
  build_projection(P, o);
  Problem& Q = problem_of(P.proj);
  const int64_t npde = pde_points(P);
  const int K = P.ncomp;
  std::vector<double> val = [&] {
    std::vector<double> v((size_t)npde * K);
    if (is_device_ptr(values))
      RFM_HIP(hipMemcpy(v.data(), values, v.size() * 8, hipMemcpyDeviceToHost));
    else
      std::copy(values, values + v.size(), v.begin());
    return v;
  }();
  for (double x : val) RFM_CHECK(std::isfinite(x), RFM_ENUMERIC, "rfm_project: non-finite values");
  // row data of Q in its row order: per PDE group, per equation (component) k, per point
  std::vector<double> rd;
  rd.reserve((size_t)Q.m);
  int64_t base = 0;
  for (const auto& g : P.groups) {
    if (g.kind != RFM_PDE || g.npts == 0) continue;
    for (int k = 0; k < K; ++k)
      for (int64_t q = 0; q < g.npts; ++q) rd.push_back(val[(size_t)(base + q) * K + k]);
    base += g.npts;
  }
  RFM_CHECK((int64_t)rd.size() == Q.m, RFM_EINVAL, "internal: projection rows");
  Q.rowdata = rd;
  RFM_HIP(hipMemcpyAsync(Q.d_rowdata.p, rd.data(), rd.size() * 8, hipMemcpyHostToDevice, Q.stream));
  // D F(0) = -D f (Phi and D do not change)
  RFM_HIP(hipMemsetAsync(Q.d_u.p, 0, Q.n * sizeof(double), Q.stream));
  launch_assemble(Q, Q.d_u.p, o.row_scale_c);
  Q.d_vec.resize(6 * std::max(Q.m, Q.n));
  double* rhs = Q.d_vec.p + 5 * std::max(Q.m, Q.n);
  launch_neg_mul(Q, Q.m, nullptr, Q.d_DF.p, rhs);
  DBuf<double> y, u;
  y.resize(Q.n);
  u.resize(Q.n);
  int it = 0, is = 0;
  lsqr_run(Q, rhs, o.lsqr_tol, o.lsqr_max_iter, y.p, &it, &is);
  launch_trsv(Q, y.p, u.p, false, nullptr, nullptr, 0, 0, nullptr);
  check_trsv_error(Q);
  copy_out(Q, u_out, u.p, Q.n);
  if (resnorm) {
    double nr = 0.0;
    api_residual(Q, u.p, nullptr, &nr);
    *resnorm = nr;
  }
  RFM_HIP(hipStreamSynchronize(Q.stream));
}

// network inputs at the PDE points: (encoded params, x) per point, X [npde][nparam + dim]; with lo and hi
// each parameter is mapped affinely from [lo_j, hi_j] to [-1, 1]
void warm_inputs(const Problem& P, const double* params, const double* lo, const double* hi, int nparam,
                 float* X) {
  RFM_CHECK((lo == nullptr) == (hi == nullptr), RFM_EINVAL, "parameter ranges: give both lo and hi, or neither");
  std::vector<double> enc(nparam);
  for (int j = 0; j < nparam; ++j) {
    RFM_CHECK(std::isfinite(params[j]), RFM_ENUMERIC, "non-finite parameter");
    if (lo) {
      RFM_CHECK(std::isfinite(lo[j]) && std::isfinite(hi[j]) && hi[j] > lo[j], RFM_EINVAL,
                "parameter ranges need finite lo < hi");
      enc[j] = 2.0 * (params[j] - lo[j]) / (hi[j] - lo[j]) - 1.0;
    } else {
      enc[j] = params[j];
    }
  }
  const int in_dim = nparam + P.dim;
  int64_t k = 0;
  for (const auto& g : P.groups) {
    if (g.kind != RFM_PDE) continue;
    for (int64_t q = 0; q < g.npts; ++q, ++k) {
      for (int j = 0; j < nparam; ++j) X[k * in_dim + j] = (float)enc[j];
      for (int a = 0; a < P.dim; ++a) X[k * in_dim + nparam + a] = (float)P.px[(g.pt0 + q) * P.dim + a];
    }
  }
}

}  // namespace

}  // namespace rfm

using namespace rfm;

extern "C" {

int64_t rfm_num_pde_points(rfm_problem* p) {
  if (!p) return -1;
  return pde_points(problem_of(p));
}

rfm_status rfm_get_pde_points(rfm_problem* p, double* x, int32_t* owner) {
  return guarded([&] {
    RFM_CHECK(p != nullptr, RFM_EINVAL, "null problem");
    const Problem& P = problem_of(p);
    int64_t k = 0;
    for (const auto& g : P.groups) {
      if (g.kind != RFM_PDE) continue;
      for (int64_t q = 0; q < g.npts; ++q, ++k) {
        if (x)
          for (int a = 0; a < P.dim; ++a) x[k * P.dim + a] = P.px[(g.pt0 + q) * P.dim + a];
        if (owner) owner[k] = g.owner;
      }
    }
  });
}

rfm_status rfm_project(rfm_problem* p, const rfm_solve_opts* opts, const double* values, double* u_out,
                       double* resnorm) {
  return guarded([&] {
    RFM_CHECK(p && opts && values && u_out, RFM_EINVAL, "rfm_project: NULL argument");
    RFM_CHECK(opts->sketch_factor > 1.0 && opts->lsqr_tol > 0 && opts->lsqr_max_iter >= 1 && opts->row_scale_c > 0,
              RFM_EINVAL, "rfm_project: bad options");
    Problem& P = problem_of(p);
    RFM_HIP(hipSetDevice(P.device));
    check(rfm_finalize(p));
    project(P, *opts, values, u_out, resnorm);
  });
}

rfm_status rfm_warm_inputs(rfm_problem* p, const double* params, const double* param_lo, const double* param_hi,
                           int32_t nparam, float* X) {
  return guarded([&] {
    RFM_CHECK(p && X && nparam >= 0 && (params || nparam == 0), RFM_EINVAL, "rfm_warm_inputs: bad argument");
    Problem& P = problem_of(p);
    check(rfm_finalize(p));
    const int64_t npde = pde_points(P);
    std::vector<float> h((size_t)npde * (nparam + P.dim));
    warm_inputs(P, params, param_lo, param_hi, nparam, h.data());
    if (is_device_ptr(X)) {
      RFM_HIP(hipSetDevice(P.device));
      RFM_HIP(hipMemcpy(X, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
      std::copy(h.begin(), h.end(), X);
    }
  });
}

rfm_status rfm_warm_start(rfm_problem* p, rfm_mlp* net, const rfm_solve_opts* opts, const double* params,
                          const double* param_lo, const double* param_hi, int32_t nparam, double* u_out,
                          double* info) {
  return guarded([&] {
    RFM_CHECK(p && net && opts && u_out && nparam >= 0 && (params || nparam == 0), RFM_EINVAL,
              "rfm_warm_start: NULL argument");
    Problem& P = problem_of(p);
    RFM_HIP(hipSetDevice(P.device));
    check(rfm_finalize(p));
    const int in_dim = nparam + P.dim;
    const int64_t npde = pde_points(P);
    RFM_CHECK(npde > 0, RFM_EINVAL, "rfm_warm_start: the problem has no PDE points");
    // the network's shape must match (params, x) -> ncomp values
    std::vector<float> X((size_t)npde * in_dim);
    warm_inputs(P, params, param_lo, param_hi, nparam, X.data());
    mlp_check_shape(net, in_dim, P.ncomp);
    std::vector<float> Y((size_t)npde * P.ncomp);
    check(rfm_mlp_predict(net, X.data(), npde, Y.data()));
    std::vector<double> val(Y.begin(), Y.end());
    std::vector<double> uw((size_t)P.n), zero((size_t)P.n, 0.0);
    project(P, *opts, val.data(), uw.data(), nullptr);
    // the solver's merit ||D F|| with one row scale for both candidates: D0, the scale at u = 0
    P.d_F0.resize(P.m);
    RFM_HIP(hipMemsetAsync(P.d_u.p, 0, P.n * sizeof(double), P.stream));
    launch_assemble(P, P.d_u.p, opts->row_scale_c);
    P.have_J = true;
    P.have_J32 = false;
    P.pan_prec = -1;
    P.cur_c = opts->row_scale_c;
    launch_diff_norm2(P, P.m, P.d_DF.p, nullptr, nullptr, P.d_scal.p);
    const double r0 = std::sqrt(read_scalar(P, P.d_scal.p));
    copy_in(P, P.d_u.p, uw.data(), P.n);
    launch_row_eval(P, P.d_u.p, nullptr, P.d_lsab.p);
    launch_residual_from_ab(P, P.d_lsab.p, P.d_F0.p, P.d_scal.p + 1);
    launch_diff_norm2(P, P.m, P.d_F0.p, nullptr, P.d_D.p, P.d_scal.p);
    const double rw = std::sqrt(read_scalar(P, P.d_scal.p));
    const bool keep = std::isfinite(rw) && rw < r0;
    if (is_device_ptr(u_out))
      RFM_HIP(hipMemcpy(u_out, keep ? uw.data() : zero.data(), P.n * 8, hipMemcpyHostToDevice));
    else
      std::copy((keep ? uw : zero).begin(), (keep ? uw : zero).end(), u_out);
    if (info) {
      info[0] = rw;
      info[1] = r0;
      info[2] = keep ? 1.0 : 0.0;
    }
  });
}

}  // extern "C"
