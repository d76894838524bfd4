// Newton drivers: IPN (Alg. 1) and AMIPN (Alg. 2), the golden-section line
// search, and the remaining C-ABI calls (solve, residual, eval, line search).
//
// Readings where the paper is silent: the row scale is recomputed at every
// Jacobian evaluation and frozen for the LSQR solves, line searches and stop
// tests that use that Jacobian; the full step is accepted when it lowers
// ||D F|| by the factor (1 - 1e-4), otherwise a golden-section search on [0, 1]
// returns the evaluated step with the smallest ||D F|| (ties to the larger
// step) and a step is only taken when it lowers ||D F||.
#include <chrono>
#include <cmath>
#include <cstring>

#include "rfm_internal.h"

namespace rfm {

double read_scalar(Problem& P, const double* d) {
  double h = 0.0;
  RFM_HIP(hipMemcpyAsync(&h, d, sizeof(double), hipMemcpyDeviceToHost, P.stream));
  RFM_HIP(hipStreamSynchronize(P.stream));
  return h;
}

namespace {

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Driver {
  Problem& P;
  rfm_solve_opts o;
  rfm_solve_stats st{};
  int jac_index = 0;
  double* ab = nullptr;  // line-search products [m][2 + 2K]
  // copy of D J used by LSQR: the FP32 copy while it works, FP64 from the first
  // FP32 step that fails (LSQR at its iteration limit, or no decrease in the line
  // search), for the rest of the solve
  int lsqr_prec = RFM_PREC_F64;

  Driver(Problem& p, const rfm_solve_opts& opts)
      : P(p), o(opts), jac_index(opts.jac_index0), lsqr_prec(opts.lsqr_prec) {
    ab = P.d_lsab.p;
    P.verbose = opts.verbose;
  }
  ~Driver() { P.verbose = 0; }

  void sync() { RFM_HIP(hipStreamSynchronize(P.stream)); }

  // J, D, R at u (Alg. 1 step 2); returns false if R does not exist
  void precondition(const double* u) {
    double t0 = now();
    launch_assemble(P, u, o.row_scale_c);
    P.have_J = true;
    P.have_J32 = false;
    P.pan_prec = -1;
    P.cur_c = o.row_scale_c;
    if (lsqr_prec == RFM_PREC_F32) launch_cast_f32(P);
    sync();
    double t1 = now();
    P.s = (int64_t)std::ceil(o.sketch_factor * (double)P.n);
    if (o.sketch_rows_per_pass > 0 || qr_should_stream(P)) {
      // B is produced and folded into R a block of rows at a time
      P.have_B = false;
      P.have_R = false;
      const int64_t rpp = std::max(0, o.sketch_rows_per_pass);
      const double t_sk =
          o.sketch_kind == RFM_SKETCH_COUNT
              ? streamed_count_sketch_qr(P, o.sketch_seed, (uint64_t)jac_index, rpp)
              : streamed_sketch_qr(P, o.sketch_seed, (uint64_t)jac_index, o.sketch_prec, o.sketch_pieces, rpp);
      P.have_R = true;
      double t3 = now();
      st.t_assemble += t1 - t0;
      st.t_sketch += t_sk;
      st.t_qr += (t3 - t1) - t_sk;
      ++jac_index;
      ++st.jac_evals;
      return;
    }
    if (o.sketch_kind == RFM_SKETCH_COUNT)
      launch_count_sketch(P, o.sketch_seed, (uint64_t)jac_index);
    else if (o.sketch_prec == RFM_PREC_F64)
      launch_sketch(P, o.sketch_seed, (uint64_t)jac_index, o.sketch_prec);
    else
      launch_sketch_lowp(P, o.sketch_seed, (uint64_t)jac_index, o.sketch_prec, o.sketch_pieces);
    sync();
    double t2 = now();
    P.have_B = true;
    P.have_R = false;
    qr_factor(P);  // throws RFM_ESINGULAR
    P.have_B = false;
    P.have_R = true;
    double t3 = now();
    st.t_assemble += t1 - t0;
    st.t_sketch += t2 - t1;
    st.t_qr += t3 - t2;
    ++jac_index;
    ++st.jac_evals;
  }

  // unscaled F(z) into F, and ||D F(z)||
  double residual(const double* z, double* F) {
    launch_row_eval(P, z, nullptr, ab);
    launch_residual_from_ab(P, ab, F, P.d_scal.p + 1);
    launch_diff_norm2(P, P.m, F, nullptr, P.d_D.p, P.d_scal.p);
    return std::sqrt(read_scalar(P, P.d_scal.p));
  }

  // direction d = R^{-1} LSQR(D J R^{-1}, -D F); returns LSQR's stop rule
  int direction(const double* F, double* d, double* y) {
    double t0 = now();
    double* rhs = P.d_F1.p + P.m;  // second half of the scratch
    launch_neg_mul(P, P.m, P.d_D.p, F, rhs);
    int it = 0, is = 0;
    lsqr_run(P, rhs, o.lsqr_tol, o.lsqr_max_iter, y, &it, &is, lsqr_prec);
    launch_trsv(P, y, d, false, nullptr, nullptr, 0, 0, nullptr);
    check_trsv_error(P);
    st.t_lsqr += now() - t0;
    st.lsqr_iters_total += it;
    if (st.nsteps < RFM_MAX_STEPS) st.lsqr_iters[st.nsteps] += it;
    return is;
  }

  void leave_fp32() {
    lsqr_prec = RFM_PREC_F64;
    st.lsqr_fp64_fallback = 1;
    if (o.verbose) std::fprintf(stderr, "[rfm] FP32 LSQR operator abandoned: continuing with FP64\n");
  }

  // Newton direction and golden-section step from z (phi0 = ||D F(z)||): returns alpha (0: no decrease)
  double step(double* z, const double* F, double* d, double* y, double phi0, double* phi1) {
    if (st.nsteps < RFM_MAX_STEPS) st.lsqr_iters[st.nsteps] = 0;
    int is = direction(F, d, y);
    if (lsqr_prec == RFM_PREC_F32 && is == 0) {
      leave_fp32();
      is = direction(F, d, y);
    }
    double alpha = linesearch(z, d, phi0, o.gs_iters, phi1);
    if (alpha == 0.0 && lsqr_prec == RFM_PREC_F32) {
      leave_fp32();
      direction(F, d, y);
      alpha = linesearch(z, d, phi0, o.gs_iters, phi1);
    }
    return alpha;
  }

  double phi(double alpha) {
    launch_phi(P, ab, alpha, P.d_D.p, P.d_scal.p);
    return std::sqrt(read_scalar(P, P.d_scal.p));
  }

  // golden-section search on phi(a) = ||D F(z + a d)||; returns a (0: no decrease) and phi(a)
  double linesearch(const double* z, const double* d, double phi0, int gs_iters, double* phi_out) {
    double t0 = now();
    launch_row_eval(P, z, d, ab);
    const double accept = 1e-4;
    const double G = (std::sqrt(5.0) - 1.0) / 2.0;
    double f1 = phi(1.0);
    double best_a = 1.0, best_f = f1;
    if (!(f1 <= (1.0 - accept) * phi0)) {
      auto consider = [&](double a, double f) {
        if (f < best_f || (f == best_f && a > best_a)) {
          best_a = a;
          best_f = f;
        }
      };
      double a = 0.0, b = 1.0;
      double c = b - G * (b - a), dd = a + G * (b - a);
      double fc = phi(c), fd = phi(dd);
      consider(c, fc);
      consider(dd, fd);
      for (int it = 0; it < gs_iters; ++it) {
        if (fc < fd) {
          b = dd;
          dd = c;
          fd = fc;
          c = b - G * (b - a);
          fc = phi(c);
          consider(c, fc);
        } else {
          a = c;
          c = dd;
          fc = fd;
          dd = a + G * (b - a);
          fd = phi(dd);
          consider(dd, fd);
        }
      }
      if (!(best_f < phi0)) {
        best_a = 0.0;
        best_f = phi0;
      }
    }
    st.t_linesearch += now() - t0;
    *phi_out = best_f;
    return best_a;
  }

  // one outer step: the directions it computed and its Flag (1: fresh J, D, R for the next one)
  void log_outer(int inner, bool flag) {
    if (st.outer_iters < RFM_MAX_STEPS) {
      st.inner_steps[st.outer_iters] = inner;
      st.flags[st.outer_iters] = flag ? 1 : 0;
    }
    ++st.outer_iters;
  }

  void log_step(double alpha, double resn) {
    if (st.nsteps < RFM_MAX_STEPS) {
      st.alphas[st.nsteps] = alpha;
      st.resnorms[st.nsteps] = resn;
    }
    ++st.nsteps;
    if (o.verbose)
      std::fprintf(stderr, "[rfm] step %d NJ %d lsqr %d alpha %.6g ||DF|| %.6e\n", st.nsteps, st.jac_evals,
                   st.nsteps <= RFM_MAX_STEPS ? st.lsqr_iters[st.nsteps - 1] : -1, alpha, resn);
  }

  rfm_status ipn(double* u) {
    double* du = P.d_du.p;
    double* y = P.d_vec.p;
    for (int k = 0; k < o.max_outer; ++k) {
      precondition(u);
      double* F = P.d_F0.p;
      const double phi0 = residual(u, F);
      if (phi0 == 0.0) {
        st.final_resnorm = 0.0;
        return RFM_OK;
      }
      double phi1 = 0.0;
      const double alpha = step(u, F, du, y, phi0, &phi1);
      log_outer(1, true);
      if (alpha == 0.0) {
        log_step(0.0, phi0);
        st.final_resnorm = phi0;
        return RFM_ESTALL;
      }
      launch_axpy(P, P.n, alpha, du, u);
      log_step(alpha, phi1);
      st.final_resnorm = phi1;
      if (std::fabs(phi1 - phi0) < o.outer_tol || phi1 == 0.0) return RFM_OK;
    }
    return RFM_ENOCONV;
  }

  rfm_status amipn(double* u) {
    double* z = P.d_vec.p + 2 * std::max(P.m, P.n);
    double* d = P.d_du.p;
    double* y = P.d_vec.p;
    double* Fz = P.d_F0.p;
    double* Fn = P.d_F1.p;
    precondition(u);
    bool fresh = true;
    for (int k = 0; k < o.max_outer; ++k) {
      RFM_HIP(hipMemcpyAsync(z, u, P.n * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
      const double F0 = residual(z, Fz);
      const double phi_u = F0;
      if (F0 == 0.0) {
        st.final_resnorm = 0.0;
        return RFM_OK;
      }
      bool flag = true, stalled = false;
      int i = 0;
      double phiz = F0;
      for (i = 0; i < o.m_max; ++i) {
        double phin = 0.0;
        const double alpha = step(z, Fz, d, y, phiz, &phin);
        if (alpha == 0.0) {
          stalled = true;
          log_step(0.0, phiz);
          break;
        }
        launch_axpy(P, P.n, alpha, d, z);
        const double pn = residual(z, Fn);
        log_step(alpha, pn);
        launch_diff_norm2(P, P.m, Fn, Fz, P.d_D.p, P.d_scal.p);
        const double dn = std::sqrt(read_scalar(P, P.d_scal.p));
        std::swap(Fz, Fn);
        phiz = pn;
        if (dn < o.tau_rel * F0) {
          flag = false;
          break;
        }
      }
      const int inner = std::min(i + 1, o.m_max);
      if (stalled && i == 0 && fresh) {
        log_outer(inner, true);
        st.final_resnorm = phi_u;
        return RFM_ESTALL;
      }
      if (stalled) flag = true;
      log_outer(inner, flag);
      const double phi_new = phiz;
      const bool done = std::fabs(phi_new - phi_u) < o.outer_tol || phi_new == 0.0;
      RFM_HIP(hipMemcpyAsync(u, z, P.n * sizeof(double), hipMemcpyDeviceToDevice, P.stream));
      st.final_resnorm = phi_new;
      if (done && !stalled) return RFM_OK;
      if (flag) {
        precondition(u);
        fresh = true;
      } else {
        fresh = false;
      }
    }
    return RFM_ENOCONV;
  }
};

void check_opts(const rfm_solve_opts& o) {
  RFM_CHECK(o.method == RFM_IPN || o.method == RFM_AMIPN, RFM_EINVAL, "opts.method must be IPN or AMIPN");
  RFM_CHECK(o.sketch_factor > 1.0 && std::isfinite(o.sketch_factor), RFM_EINVAL, "opts.sketch_factor must be > 1");
  RFM_CHECK(o.lsqr_tol > 0 && o.lsqr_max_iter >= 1, RFM_EINVAL, "opts: bad LSQR settings");
  RFM_CHECK(o.outer_tol >= 0 && o.max_outer >= 1, RFM_EINVAL, "opts: bad outer settings");
  RFM_CHECK(o.m_max >= 1 && o.tau_rel >= 0, RFM_EINVAL, "opts: bad AMIPN settings");
  RFM_CHECK(o.row_scale_c > 0 && o.gs_iters >= 0 && o.gs_iters <= 200, RFM_EINVAL, "opts: bad scale/line search");
  RFM_CHECK(o.sketch_prec == RFM_PREC_F64 || o.sketch_prec == RFM_PREC_BF16 || o.sketch_prec == RFM_PREC_FP8,
            RFM_EINVAL, "opts.sketch_prec must be F64, BF16 or FP8");
  RFM_CHECK(o.sketch_pieces >= 0 && o.sketch_pieces <= kMaxPieces, RFM_EINVAL, "opts.sketch_pieces must be 0..16");
  RFM_CHECK(o.sketch_kind == RFM_SKETCH_GAUSSIAN || o.sketch_kind == RFM_SKETCH_COUNT, RFM_EINVAL,
            "opts.sketch_kind must be GAUSSIAN or COUNT");
  RFM_CHECK(o.sketch_kind == RFM_SKETCH_GAUSSIAN || o.sketch_prec == RFM_PREC_F64, RFM_EINVAL,
            "the count sketch is formed in FP64 (its entries are signed copies of D J)");
  RFM_CHECK(o.lsqr_prec == RFM_PREC_F64 || o.lsqr_prec == RFM_PREC_F32, RFM_EINVAL,
            "opts.lsqr_prec must be F64 or F32");
  RFM_CHECK(o.jac_index0 >= 0, RFM_EINVAL, "opts.jac_index0 must be >= 0");
}

}  // namespace

}  // namespace rfm

using namespace rfm;

extern "C" {

void rfm_solve_opts_default(rfm_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->method = RFM_IPN;
  o->sketch_factor = 3.0;
  o->sketch_seed = 1;
  o->lsqr_tol = 1e-6;
  o->lsqr_max_iter = 500;
  o->outer_tol = 1e-10;
  o->max_outer = 30;
  o->m_max = 3;
  o->tau_rel = 1e-3;
  o->row_scale_c = 100.0;
  o->gs_iters = 25;
  o->sketch_prec = RFM_PREC_F64;
  o->lsqr_prec = RFM_PREC_F64;
  o->sketch_pieces = 0;
  o->sketch_kind = RFM_SKETCH_GAUSSIAN;
  o->verbose = 0;
  o->sketch_rows_per_pass = 0;
  o->jac_index0 = 0;
}

}  // extern "C"

namespace rfm {

rfm_status api_solve(Problem& P, const rfm_solve_opts* opts, double* u_inout, rfm_solve_stats* stats) {
  RFM_CHECK(opts && u_inout, RFM_EINVAL, "rfm_solve: NULL argument");
  check_opts(*opts);
  P.d_F0.resize(P.m);
  P.d_F1.resize(2 * P.m);
  const double t0 = now();
  copy_in(P, P.d_u.p, u_inout, P.n);
  Driver D(P, *opts);
  rfm_status rc = opts->method == RFM_AMIPN ? D.amipn(P.d_u.p) : D.ipn(P.d_u.p);
  copy_out(P, u_inout, P.d_u.p, P.n);
  RFM_HIP(hipStreamSynchronize(P.stream));
  D.st.t_total = now() - t0;
  D.st.status_detail = rc;
  if (stats) *stats = D.st;
  return rc;
}

}  // namespace rfm

namespace rfm {

rfm_status api_residual(Problem& P, const double* u, double* F, double* norm) {
  P.d_F0.resize(P.m);
  copy_in(P, P.d_u.p, u, P.n);
  launch_row_eval(P, P.d_u.p, nullptr, P.d_lsab.p);
  launch_residual_from_ab(P, P.d_lsab.p, P.d_F0.p, P.d_scal.p);
  if (F) copy_out(P, F, P.d_F0.p, P.m);
  const double ss = read_scalar(P, P.d_scal.p);
  if (norm) *norm = std::sqrt(ss);
  RFM_CHECK(std::isfinite(ss), RFM_ENUMERIC, "non-finite residual");
  return RFM_OK;
}

rfm_status api_eval(Problem& P, const double* u, int64_t npts, const double* x, const int32_t* owner, int what,
                    double* out) {
  RFM_CHECK(npts >= 0 && (npts == 0 || (x && owner && out)), RFM_EINVAL, "rfm_eval: bad arguments");
  RFM_CHECK(what == RFM_EVAL_VALUE || what == RFM_EVAL_GRAD, RFM_EINVAL, "rfm_eval: what must be VALUE or GRAD");
  const int64_t per = what == RFM_EVAL_GRAD ? (int64_t)P.ncomp * P.dim : P.ncomp;
  if (npts == 0) return RFM_OK;
  copy_in(P, P.d_u.p, u, P.n);
  // owners are checked on the host before any device work
  std::vector<int32_t> own(npts);
  if (is_device_ptr(owner))
    RFM_HIP(hipMemcpy(own.data(), owner, npts * 4, hipMemcpyDeviceToHost));
  else
    std::memcpy(own.data(), owner, npts * 4);
  for (int64_t i = 0; i < npts; ++i)
    RFM_CHECK(own[i] >= 0 && own[i] < P.geom.nbox, RFM_EINVAL, "rfm_eval: owner out of range");
  DBuf<double> dx, dout;
  DBuf<int32_t> dow;
  dx.resize((size_t)npts * P.dim);
  dout.resize((size_t)(npts * per));
  dow.resize(npts);
  copy_in(P, dx.p, x, (size_t)npts * P.dim);
  RFM_HIP(hipMemcpyAsync(dow.p, own.data(), npts * 4, hipMemcpyHostToDevice, P.stream));
  launch_eval_points(P, P.d_u.p, npts, dx.p, dow.p, dout.p, what == RFM_EVAL_GRAD);
  copy_out(P, out, dout.p, (size_t)(npts * per));
  RFM_HIP(hipStreamSynchronize(P.stream));
  return RFM_OK;
}

rfm_status api_linesearch(Problem& P, const double* u, const double* du, int gs_iters, double* alpha,
                          double* phi) {
  RFM_CHECK(P.have_J, RFM_EINVAL, "line search needs an assembled Jacobian (for its row scale)");
  RFM_CHECK(u && du && alpha && phi && gs_iters >= 0, RFM_EINVAL, "rfm_stage_linesearch: bad arguments");
  copy_in(P, P.d_u.p, u, P.n);
  copy_in(P, P.d_du.p, du, P.n);
  rfm_solve_opts o;
  rfm_solve_opts_default(&o);
  Driver D(P, o);
  P.d_F0.resize(P.m);
  const double phi0 = D.residual(P.d_u.p, P.d_F0.p);
  *alpha = D.linesearch(P.d_u.p, P.d_du.p, phi0, gs_iters, phi);
  return RFM_OK;
}

}  // namespace rfm
